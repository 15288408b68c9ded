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

template <int AK, bool RMS, int EPI, bool Q, int R>
__device__ void gemm_phase(const GemmArgs& a, float4* smem4, float* rstd) {
  __shared__ float rmul[kMBq];
  if (Q) {
    // tiles in row-tile-major order: a block re-stages A only when its next
    // tile starts a new row tile
    const int ct = qgemm_col_tiles(a.N, EPI), rt = qgemm_row_tiles(a.M, R);
    int staged = -1;
    for (int t = blockIdx.x; t < ct * rt; t += gridDim.x) {
      const int r = t / ct;
      gemm_tile_q_any<AK, RMS, EPI, R>(a, t % ct, r, reinterpret_cast<uint8_t*>(smem4), rstd,
                                       rmul, r != staged);
      staged = r;
    }
    return;
  }
  const int ct = gemm_col_tiles(a.N, EPI), rt = gemm_row_tiles(a.M);
  for (int t = blockIdx.x; t < ct * rt; t += gridDim.x)
    gemm_tile_any<AK, RMS, EPI>(a, t % ct, t / ct, smem4, rstd);
}

template <int DH>
__device__ void attn_phase(const AttnArgs& a, float* smem) {
  const int groups = (a.M * a.heads + kWaves - 1) / kWaves;
  for (int g = blockIdx.x; g < groups; g += gridDim.x)
    attn_item<DH>(a, g * kWaves + (threadIdx.x >> 6), true, smem);
}

__device__ void symbol_phase(const SymArgs& c) {
  const long n = (long)c.M * c.C;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    gather_item(c.ysrc, c.src_compact, c.gpos, c.C, c.ydec, i);
    bits_item(c.gpos, c.C, c.ydec, c.mean, c.scale, c.bits, i);
  }
}

// Q: the model's projections run on MFMA (BF16/FP8) rather than FP32 SIMT;
// one instance per arithmetic keeps each one's register budget separate.
template <bool Q, int DH, int R>
__global__ void __launch_bounds__(kThreads) k_persistent(PersistArgs P) {
  extern __shared__ float4 smem4[];
  __shared__ float rstd[kMBq];
  float* smem = reinterpret_cast<float*>(smem4);
  const int L = P.L, ng = 6 + 4 * L, na = 1 + L;
  unsigned target = 0;
  int nsync = 0;
#define PSWA_SYNC                                                                  \
  if (!grid_barrier(P.bar, target, P.abort_flag, P.spin_limit)) return;            \
  if (P.trace && blockIdx.x == 0 && threadIdx.x == 0 && nsync < P.trace_len)       \
    P.trace[nsync] = wall_clock64();                                              \
  ++nsync;

  for (int t = P.t_begin; t < P.t_end; ++t) {
    const SymArgs& sy = P.stab[t];
    if (sy.M == 0) continue;  // same for every block
    const GemmArgs* g = P.gtab + (size_t)t * ng;
    const AttnArgs* at = P.atab + (size_t)t * na;

    gemm_phase<A_FLOAT, true, EPI_STORE, Q, R>(g[0], smem4, rstd);
    PSWA_SYNC
    attn_phase<DH>(at[0], smem);
    PSWA_SYNC
    gemm_phase<A_FLOAT, false, EPI_RESID, Q, R>(g[1], smem4, rstd);
    PSWA_SYNC
    for (int l = 0; l < L; ++l) {
      gemm_phase<A_FLOAT, true, EPI_QKV, Q, R>(g[2 + 4 * l], smem4, rstd);
      PSWA_SYNC
      attn_phase<DH>(at[1 + l], smem);
      PSWA_SYNC
      gemm_phase<A_FLOAT, false, EPI_RESID, Q, R>(g[3 + 4 * l], smem4, rstd);
      PSWA_SYNC
      gemm_phase<A_FLOAT, true, EPI_SWIGLU, Q, R>(g[4 + 4 * l], smem4, rstd);
      PSWA_SYNC
      gemm_phase<A_FLOAT, false, EPI_RESID, Q, R>(g[5 + 4 * l], smem4, rstd);
      PSWA_SYNC
    }
    gemm_phase<A_FLOAT, true, EPI_SILU, Q, R>(g[2 + 4 * L], smem4, rstd);
    PSWA_SYNC
    gemm_phase<A_FLOAT, false, EPI_HEAD, Q, R>(g[3 + 4 * L], smem4, rstd);
    PSWA_SYNC
    symbol_phase(sy);
    PSWA_SYNC
    gemm_phase<A_INT, false, EPI_STORE, Q, R>(g[4 + 4 * L], smem4, rstd);
    PSWA_SYNC
    gemm_phase<A_FLOAT, true, EPI_STORE, Q, R>(g[5 + 4 * L], smem4, rstd);
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

// The instance for a model: projection arithmetic, head size and (for
// BF16/FP8) the row-tile height.
const void* persistent_fn(int prec, int dh, int rtile) {
#define PSWA_P(Q_, D_, R_)                                                    \
  if (bool(prec) == Q_ && dh == D_ && (!Q_ || rtile == R_))                   \
  return reinterpret_cast<const void*>(&k_persistent<Q_, D_, R_>)
  PSWA_P(false, 16, 32); PSWA_P(false, 32, 32); PSWA_P(false, 48, 32); PSWA_P(false, 64, 32);
  PSWA_P(true, 16, 16); PSWA_P(true, 32, 16); PSWA_P(true, 48, 16); PSWA_P(true, 64, 16);
  PSWA_P(true, 16, 32); PSWA_P(true, 32, 32); PSWA_P(true, 48, 32); PSWA_P(true, 64, 32);
#undef PSWA_P
  return nullptr;
}

int persistent_max_grid(const NetDims& x, int prec) {
  const void* fn = persistent_fn(prec, x.dh, kMBq);
  if (!fn || !allow_big_lds(fn)) return 0;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kThreads,
                                                   persistent_lds_bytes(x, prec)) != hipSuccess)
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
    for (int q = 0; q < 2; ++q)
      for (int d : {16, 32, 48, 64})
        for (int r : {16, 32})
          if (const void* f = persistent_fn(q, d, r)) ok = allow_big_lds(f) && ok;
    return ok;
  }();
  (void)attr;
  void* args[] = {const_cast<PersistArgs*>(&P)};
  (void)hipLaunchKernel(fn, dim3(grid), dim3(kThreads), args, persistent_lds_bytes(x, prec), s);
}

}  // namespace pswa
