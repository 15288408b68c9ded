// Per-launch FP32 kernels of the wavefront context model for gfx950.
//
// Each kernel is a thin grid over a shared device function (device_ops.h):
// a GEMM launch is a grid of GEMM tiles, an attention launch a grid of
// (row, head) items. The same functions run inside the persistent decode
// kernel, so every path computes a row the same way.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#include "device_ops.h"
#include "mfma_ops.h"
#include "pswa_internal.h"

namespace pswa {

using namespace dev;

namespace {

template <int AK, bool RMS, int EPI, int KC>
__global__ void __launch_bounds__(kThreads) k_gemm(GemmArgs a) {
  extern __shared__ float4 smem4[];
  __shared__ float rstd[kMB];
  gemm_tile<AK, RMS, EPI, KC>(a, blockIdx.x, blockIdx.y, smem4, rstd);
}

template <int AK, bool RMS, int EPI, int PREC, int R, int CB>
__global__ void __launch_bounds__(kThreads) k_gemm_qb(GemmArgs a) {
  extern __shared__ float4 smem4[];
  __shared__ float rstd[R], rmul[R];
  gemm_tile_qb<AK, RMS, EPI, PREC, R, CB>(a, blockIdx.x, blockIdx.y,
                                          reinterpret_cast<uint8_t*>(smem4), rstd, rmul);
}

template <int AK, bool RMS, int EPI>
__global__ void __launch_bounds__(kThreads) k_gemm_q(GemmArgs a) {
  extern __shared__ float4 smem4[];
  __shared__ float rstd[kMBq], rmul[kMBq];
  gemm_tile_q_any<AK, RMS, EPI>(a, blockIdx.x, blockIdx.y, reinterpret_cast<uint8_t*>(smem4),
                                rstd, rmul);
}

// One wave per (row, head pair); KV16: BF16 key/value caches.
template <int DH, bool KV16>
__global__ void __launch_bounds__(kThreads) k_attn(AttnArgs a) {
  attn_item<DH, KV16>(a, blockIdx.x * kWaves + (threadIdx.x >> 6));
}

// The accumulator's null key and value as row `row` of its cache (BF16 when
// kv16), so that attention reads the null slot like any other key.
__global__ void k_null_row(float* acc_kv, size_t row, const float* knull, const float* vnull,
                           int d, int kv16) {
  for (int i = threadIdx.x; i < 2 * d; i += blockDim.x) {
    const float v = i < d ? knull[i] : vnull[i - d];
    const size_t o = row * 2 * d + i;
    if (kv16) reinterpret_cast<uint16_t*>(acc_kv)[o] = bf16_rne(v);
    else acc_kv[o] = v;
  }
}

// One block per hyperprior cell: W_h z is shared by the cell's (up to) 4x4
// positions, which differ only in their sub-position embedding.
__global__ void k_hyper_embed(const int32_t* z, int Hh, int Wh, int Ch, const float* Wm,
                              const float* P4, int H, int W, int d, float* h) {
  const int ci = blockIdx.x / Wh, cj = blockIdx.x % Wh;
  const int32_t* zr = z + (size_t)blockIdx.x * Ch;
  for (int n = threadIdx.x; n < d; n += blockDim.x) {
    const float* wr = Wm + (size_t)n * Ch;
    float acc = 0.f;
    for (int k = 0; k < Ch; ++k) acc = fmaf(float(zr[k]), wr[k], acc);
    for (int a = 0; a < 4; ++a) {
      const int i = 4 * ci + a;
      if (i >= H) break;
      for (int b = 0; b < 4; ++b) {
        const int j = 4 * cj + b;
        if (j >= W) break;
        h[((size_t)i * W + j) * d + n] = acc + P4[(a * 4 + b) * d + n];
      }
    }
  }
}

__global__ void k_gather_symbols(const int32_t* src, int compact, const int* pos, int M, int C,
                                 int32_t* ydec, int c0, int nc) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (long)M * nc) gather_item(src, compact, pos, C, ydec, idx, c0, nc);
}

// One wave per row: the sum of squares of the row's K-slice at col0, lane l
// over elements l, l + 64, ... in order, then a fixed xor tree.
__global__ void __launch_bounds__(256) k_group_rms(const float* X, int ldx, int M, int K, int col0,
                                                   const float* gain, float* Y, int ldy) {
  const int m = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (m >= M) return;
  group_rms_row(X + (size_t)m * ldx + col0, gain + col0, Y + (size_t)m * ldy + col0, K);
}

__global__ void k_symbol_bits(const int* pos, int M, int C, const int32_t* ydec,
                              const float* mean, const float* scale, float* bits) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (long)M * C) bits_item(pos, C, ydec, mean, scale, bits, idx);
}

// Fixed-order sum: thread t adds elements t, t+1024, ... with Kahan
// compensation, then a fixed LDS tree.
__global__ void __launch_bounds__(1024) k_sum(const float* v, size_t n, float* out) {
  __shared__ float sh[1024];
  float s = 0.f, comp = 0.f;
  for (size_t i = threadIdx.x; i < n; i += 1024) {
    const float y = v[i] - comp;
    const float t = s + y;
    comp = (t - s) - y;
    s = t;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

__global__ void k_cdf_select(const float* mean, const float* lsig, size_t n, float ln_smin,
                             float inv_delta, int32_t* center, uint16_t* index) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  select_table(mean[i], lsig[i], ln_smin, inv_delta, center + i, index + i);
}

// Wavefront order of all positions: step t = j + s*i, rows ascending within
// a step. Position (i, j) lands at start(t) + (i - i_lo(t)), where start(t)
// counts the positions of earlier steps and i_lo(t) is the first row on t.

inline unsigned blocks_for(long n, int t) { return unsigned((n + t - 1) / t); }

// Large-M launch of a low-precision GEMM: 128-row tiles when the staged rows
// fit (K <= 512), else 32-row tiles; 4 or 2 groups of 16 weight rows per
// wave by the width of the output.
template <int AK, bool RMS, int EPI, int PREC, int R, int CB>
void launch_big(const GemmArgs& a, hipStream_t s) {
  const void* fn = reinterpret_cast<const void*>(&k_gemm_qb<AK, RMS, EPI, PREC, R, CB>);
  static const bool attr_set = allow_big_lds(fn);
  (void)attr_set;
  dim3 grid(qgemm_big_col_tiles(a.N, EPI, CB), qgemm_row_tiles(a.M, R));
  hipLaunchKernelGGL((k_gemm_qb<AK, RMS, EPI, PREC, R, CB>), grid, dim3(kThreads),
                     qgemm_lds_bytes(a.K, PREC, R), s, a);
}

template <int AK, bool RMS, int EPI, int PREC>
void launch_big_any(const GemmArgs& a, hipStream_t s) {
  const bool tall = a.K <= 512, wide = a.N >= 1024;
  if (tall && wide) launch_big<AK, RMS, EPI, PREC, 128, 4>(a, s);
  else if (tall) launch_big<AK, RMS, EPI, PREC, 128, 2>(a, s);
  else if (wide) launch_big<AK, RMS, EPI, PREC, 32, 4>(a, s);
  else launch_big<AK, RMS, EPI, PREC, 32, 2>(a, s);
}

constexpr int kBigM = 256;  // rows from which the large tile pays

template <int AK, bool RMS, int EPI>
void launch_gemm_f32(const GemmArgs& a, hipStream_t s) {
  dim3 grid(gemm_col_tiles(a.N, EPI), gemm_row_tiles(a.M));
  const size_t lds = gemm_lds_bytes(a.K);
#define PSWA_KC(n)                                                                  \
  case n: {                                                                         \
    static const bool attr_set = allow_big_lds(                                     \
        reinterpret_cast<const void*>(&k_gemm<AK, RMS, EPI, n>));                   \
    (void)attr_set;                                                                 \
    hipLaunchKernelGGL((k_gemm<AK, RMS, EPI, n>), grid, dim3(kThreads), lds, s, a); \
    break;                                                                          \
  }
  switch (kc_for(a.K)) {
    PSWA_KC(1)
    PSWA_KC(2)
    PSWA_KC(4)
    PSWA_KC(8)
    default: break;
  }
#undef PSWA_KC
}

template <int AK, bool RMS, int EPI>
void launch_gemm(const GemmArgs& a, hipStream_t s) {
  if (a.prec != PSWA_PREC_F32 && a.M >= kBigM) {
    if (a.prec == PSWA_PREC_BF16) launch_big_any<AK, RMS, EPI, PSWA_PREC_BF16>(a, s);
    else launch_big_any<AK, RMS, EPI, PSWA_PREC_FP8>(a, s);
    return;
  }
  if (a.prec != PSWA_PREC_F32) {
    static const bool attr_set =
        allow_big_lds(reinterpret_cast<const void*>(&k_gemm_q<AK, RMS, EPI>));
    (void)attr_set;
    dim3 grid(qgemm_col_tiles(a.N, EPI), qgemm_row_tiles(a.M));
    hipLaunchKernelGGL((k_gemm_q<AK, RMS, EPI>), grid, dim3(kThreads),
                       qgemm_lds_bytes(a.K, a.prec), s, a);
    return;
  }
  launch_gemm_f32<AK, RMS, EPI>(a, s);
}

[[noreturn]] void no_instance(const char* what, int a, int b, int c) {
  std::fprintf(stderr, "pswa: no %s instance for (%d, %d, %d)\n", what, a, b, c);
  std::abort();
}

void gemm_dispatch(AKind ak, bool rms, Epi epi, const GemmArgs& a, hipStream_t s) {
#define PSWA_G(AK_, R_, E_) \
  if (ak == AK_ && rms == R_ && epi == E_) return launch_gemm<AK_, R_, E_>(a, s)
  PSWA_G(A_INT, false, EPI_STORE);
  PSWA_G(A_FLOAT, true, EPI_STORE);
  PSWA_G(A_FLOAT, false, EPI_STORE);
  PSWA_G(A_FLOAT, false, EPI_RESID);
  PSWA_G(A_FLOAT, true, EPI_QKV);
  PSWA_G(A_FLOAT, true, EPI_SILU);
  PSWA_G(A_FLOAT, true, EPI_SWIGLU);
  PSWA_G(A_FLOAT, false, EPI_HEAD);
#undef PSWA_G
  // symbols of earlier channel groups added to the channel transformer's
  // stream (FP32 in every precision)
  if (ak == A_INT && !rms && epi == EPI_RESID && a.prec == PSWA_PREC_F32)
    return launch_gemm_f32<A_INT, false, EPI_RESID>(a, s);
  no_instance("GEMM", int(ak) * 10 + int(rms), int(epi), a.prec);
}

void attention_dispatch(const AttnArgs& a, hipStream_t s) {
  const dim3 grid(blocks_for((long)a.M * attn_pairs(a.heads), kWaves));
#define PSWA_ATTN(D_)                                                                    \
  case D_:                                                                               \
    if (a.kv16) hipLaunchKernelGGL((k_attn<D_, true>), grid, dim3(kThreads), 0, s, a);   \
    else hipLaunchKernelGGL((k_attn<D_, false>), grid, dim3(kThreads), 0, s, a);         \
    break;
  switch (a.dh) {  // other head sizes are rejected when the model is created
    PSWA_ATTN(16)
    PSWA_ATTN(32)
    PSWA_ATTN(48)
    PSWA_ATTN(64)
    default: no_instance("attention", a.dh, 0, 0);
  }
#undef PSWA_ATTN
}

}  // namespace

bool allow_big_lds(const void* fn) {
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(kMaxDynLds)) ==
         hipSuccess;
}

double gemm_alg_bytes(const GemmArgs& a, Epi epi) {
  // weights once, A rows in, outputs (and residual / head outputs) out
  const bool paired = epi == EPI_SWIGLU || epi == EPI_HEAD;
  const double wbytes = a.prec == PSWA_PREC_BF16 ? 2.0 : a.prec == PSWA_PREC_FP8 ? 1.0 : 4.0;
  const double wmat = (paired ? 2.0 : 1.0) * a.N * a.K * wbytes;
  const double io = double(a.M) * a.K * 4.0 +
                    double(a.M) * a.N * 4.0 *
                        (epi == EPI_RESID ? 2.0 : epi == EPI_HEAD ? 4.5 : 1.0);
  return wmat + io;
}

double attn_alg_bytes(const AttnArgs& a) {
  // every slot's K and V rows (for the cyclic schedule an upper bound: the
  // step mask hides part of the window)
  const double keys = attn_slots(a);
  // K and V rows of every window slot, the query and the output
  return double(a.M) * (keys * 2.0 * a.d * (a.kv16 ? 2.0 : 4.0) + 2.0 * a.d * 4.0);
}

void gemm_run(AKind ak, bool rms, Epi epi, const GemmArgs& a, hipStream_t s) {
  if (a.M <= 0) return;
  const int ev = prof_begin(s);
  gemm_dispatch(ak, rms, epi, a, s);
  if (ev >= 0)
    prof_end(ev, s, a.role, gemm_alg_bytes(a, epi),
             2.0 * a.M * a.N * a.K * ((epi == EPI_SWIGLU || epi == EPI_HEAD) ? 2.0 : 1.0));
}

void attention_f32(const AttnArgs& a, hipStream_t s) {
  if (a.M <= 0) return;
  const int ev = prof_begin(s);
  attention_dispatch(a, s);
  if (ev >= 0) {
    const double keys = attn_slots(a);
    prof_end(ev, s, a.role, attn_alg_bytes(a), double(a.M) * a.heads * keys * 4.0 * a.dh);
  }
}

void hyper_embed(const int32_t* z, int Hh, int Wh, int Ch, const float* Wm, const float* P4,
                 int H, int W, int d, float* h, hipStream_t s) {
  const int ev = prof_begin(s);
  hipLaunchKernelGGL(k_hyper_embed, dim3(Hh * Wh), dim3(256), 0, s, z, Hh, Wh, Ch, Wm, P4, H,
                     W, d, h);
  prof_end(ev, s, R_HYPER,
           4.0 * (double(Hh) * Wh * Ch + double(d) * Ch + 16.0 * d + double(H) * W * d),
           2.0 * Hh * Wh * d * Ch);
}

void gather_symbols(const int32_t* src, int compact, const int* pos, int M, int C,
                    int32_t* ydec, hipStream_t s, int c0, int nc) {
  if (nc < 0) nc = C;
  if (M <= 0 || nc <= 0) return;
  const int ev = prof_begin(s);
  hipLaunchKernelGGL(k_gather_symbols, dim3(blocks_for((long)M * nc, 256)), dim3(256), 0, s, src,
                     compact, pos, M, C, ydec, c0, nc);
  prof_end(ev, s, R_GATHER, 8.0 * M * nc + 4.0 * M, 0.0);
}

void group_rmsnorm(const float* X, int ldx, int M, int K, int col0, const float* gain, float* Y,
                   int ldy, hipStream_t s) {
  if (M <= 0) return;
  hipLaunchKernelGGL(k_group_rms, dim3((M + 3) / 4), dim3(256), 0, s, X, ldx, M, K, col0, gain, Y,
                     ldy);
}

void null_row(float* acc_kv, size_t row, const float* knull, const float* vnull, int d, int kv16,
              hipStream_t s) {
  hipLaunchKernelGGL(k_null_row, dim3(1), dim3(256), 0, s, acc_kv, row, knull, vnull, d, kv16);
}

void symbol_bits(const int* pos, int M, int C, const int32_t* ydec, const float* mean,
                 const float* scale, float* bits, hipStream_t s) {
  if (M <= 0) return;
  const int ev = prof_begin(s);
  hipLaunchKernelGGL(k_symbol_bits, dim3(blocks_for((long)M * C, 256)), dim3(256), 0, s, pos, M,
                     C, ydec, mean, scale, bits);
  prof_end(ev, s, R_BITS, 16.0 * M * C + 4.0 * M, 0.0);
}

void sum_f32(const float* v, size_t n, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(1024), 0, s, v, n, out);
}

void cdf_select(const float* mean, const float* lsig, size_t n, float ln_smin, float inv_delta,
                int32_t* center, uint16_t* index, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_cdf_select, dim3(blocks_for((long)n, 256)), dim3(256), 0, s, mean, lsig,
                     n, ln_smin, inv_delta, center, index);
}


}  // namespace pswa
