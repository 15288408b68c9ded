// FP32 kernels of the wavefront context model for gfx950 (64-wide waves).
//
// One set of kernels serves both the parallel encode form (every position of
// the frame in one launch) and the per-diagonal decode steps: a launch gets a
// row -> position map and each output row is computed the same way whatever
// the number of rows, so encode and decode agree bit for bit.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

#include "pswa_internal.h"

namespace pswa {

namespace {

constexpr float kEps = 1e-5f;

__device__ __forceinline__ int map_row(const int* idx, int m) { return idx ? idx[m] : m; }

__device__ __forceinline__ float silu(float v) { return v / (1.0f + expf(-v)); }

// Centre and table index of one symbol, one rounding per operation (no
// contraction), so the decision equals the documented float32 formula.
__device__ __forceinline__ void select_table(float mu, float lsig, float ln_smin, float inv_delta,
                                             int32_t* c_out, uint16_t* i_out) {
#pragma clang fp contract(off)
  const float c = floorf(mu + 0.5f);
  const float ph = (mu - c) + 0.5f;
  const float m = fminf(15.0f, floorf(ph * 16.0f));
  const float t = (lsig - ln_smin) * inv_delta;
  const float s = fminf(63.0f, fmaxf(0.0f, floorf(t + 0.5f)));
  *c_out = int32_t(c);
  *i_out = uint16_t(int(s) * 16 + int(m));
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------- GEMM
// Skinny FP32 GEMM for the few rows of a diagonal (and, row group by row
// group, for a whole frame). A 256-thread block owns 16 weight rows (4 per
// wave) and up to kMB rows of A:
//   1. every wave loads its 4 weight rows into registers: lane l takes the
//      float4 chunks l, l + 64, ... (a compile-time count, all in flight);
//   2. the block stages the raw A tile [rows][K] in LDS, all loads at once;
//   3. RMSNorm rows: lane l sums x^2 over its chunks in order, then a fixed
//      xor tree gives the row's 1/rms;
//   4. each lane keeps an fmaf chain per (row, weight row) over its chunks,
//      and the 64 lane partials are summed lane 0..63 in order.
// The RMSNorm scale is applied to the finished dot product:
//   sum_k (x_k * rstd * g_k) w_k  ==  rstd * sum_k (x_k g_k) w_k.
// An output's arithmetic depends only on K, never on the number of rows in
// the launch, so encode and decode agree bit for bit.
// Paired epilogues (SwiGLU, head): a wave's weight rows are W[n], W[n+1],
// W2[n], W2[n+1] and it produces outputs n and n+1.
constexpr int kRowsW = 4;   // weight rows per wave
constexpr int kWaves = 4;
constexpr int kMB = 16;     // A rows per block

__device__ __forceinline__ float dot4(float4 x, float4 w, float acc) {
  acc = fmaf(x.x, w.x, acc);
  acc = fmaf(x.y, w.y, acc);
  acc = fmaf(x.z, w.z, acc);
  return fmaf(x.w, w.w, acc);
}

template <int AK, bool RMS, int EPI, int KC>
__global__ void __launch_bounds__(256) k_gemm(GemmArgs a) {
  constexpr bool PAIRED = (EPI == EPI_SWIGLU || EPI == EPI_HEAD);
  extern __shared__ float4 smem4[];
  float* smem = reinterpret_cast<float*>(smem4);
  __shared__ float rstd[kMB];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n0 = blockIdx.x * kWaves * (PAIRED ? 2 : kRowsW) + wave * (PAIRED ? 2 : kRowsW);
  const int m0 = blockIdx.y * kMB;
  const int K = a.K, K4 = a.K / 4;
  const int rows = min(kMB, a.M - m0);

  // 1. weight rows -> registers
  const float* wrow[kRowsW];
#pragma unroll
  for (int j = 0; j < kRowsW; ++j) {
    if (PAIRED) {
      const int n = min(n0 + (j & 1), a.N - 1);
      wrow[j] = (j < 2 ? a.W : a.W2) + (size_t)n * K;
    } else {
      wrow[j] = a.W + (size_t)min(n0 + j, a.N - 1) * K;
    }
  }
  float4 w[KC][kRowsW];
  float4 g[KC];
#pragma unroll
  for (int it = 0; it < KC; ++it) {
    const int c = lane + 64 * it;
    const bool in = c < K4;
#pragma unroll
    for (int j = 0; j < kRowsW; ++j)
      w[it][j] = in ? *reinterpret_cast<const float4*>(wrow[j] + 4 * c) : make_float4(0, 0, 0, 0);
    g[it] = make_float4(1.f, 1.f, 1.f, 1.f);
    if (RMS && in) g[it] = *reinterpret_cast<const float4*>(a.gain + 4 * c);
    if (AK == A_INT && in) g[it] = *reinterpret_cast<const float4*>(a.xscale + 4 * c);
  }

  // 2. raw A tile -> LDS (int inputs are converted, unscaled)
  for (int e = tid; e < rows * K4; e += blockDim.x) {
    const int m = e / K4, c = e % K4;
    const size_t off = (size_t)map_row(a.xrow, m0 + m) * a.ldx + 4 * c;
    float4 x;
    if (AK == A_INT) {
      const int4 xi = *reinterpret_cast<const int4*>(a.Xi + off);
      x = make_float4(float(xi.x), float(xi.y), float(xi.z), float(xi.w));
    } else {
      x = *reinterpret_cast<const float4*>(a.X + off);
    }
    smem4[m * K4 + c] = x;
  }
  __syncthreads();

  // 3. 1/rms of the tile's rows: wave w takes rows w, w+4, ...
  if (RMS) {
    for (int m = wave; m < rows; m += kWaves) {
      float ss = 0.f;
#pragma unroll
      for (int it = 0; it < KC; ++it) {
        const int c = lane + 64 * it;
        if (c < K4) {
          const float4 x = smem4[m * K4 + c];
          ss = dot4(x, x, ss);
        }
      }
      ss = wave_sum(ss);
      if (lane == 0) rstd[m] = 1.0f / sqrtf(ss / float(K) + kEps);
    }
  }

  // 4. lane partials over this lane's chunks
  float acc[kMB][kRowsW];
#pragma unroll
  for (int m = 0; m < kMB; ++m)
#pragma unroll
    for (int j = 0; j < kRowsW; ++j) acc[m][j] = 0.f;
#pragma unroll
  for (int m = 0; m < kMB; ++m) {
    if (m < rows) {
#pragma unroll
      for (int it = 0; it < KC; ++it) {
        const int c = lane + 64 * it;
        if (c < K4) {
          float4 x = smem4[m * K4 + c];
          x = make_float4(x.x * g[it].x, x.y * g[it].y, x.z * g[it].z, x.w * g[it].w);
#pragma unroll
          for (int j = 0; j < kRowsW; ++j) acc[m][j] = dot4(x, w[it][j], acc[m][j]);
        }
      }
    }
  }
  __syncthreads();  // the A tile is dead; its LDS becomes the transpose buffer

  float* red = smem + wave * (64 * 65);
#pragma unroll
  for (int m = 0; m < kMB; ++m)
#pragma unroll
    for (int j = 0; j < kRowsW; ++j) red[(m * kRowsW + j) * 65 + lane] = acc[m][j];
  __syncthreads();
  float v = 0.f;
#pragma unroll
  for (int l = 0; l < 64; ++l) v += red[lane * 65 + l];
  const int m = lane / kRowsW, j = lane % kRowsW;
  if (RMS) v *= rstd[min(m, rows - 1)];
  const int row = m0 + m;
  // paired: lanes with j = 2, 3 hold the W2 products of lanes j = 0, 1
  const float v2 = PAIRED ? __shfl(v, (lane & ~3) | ((j & 1) + 2), 64) : 0.f;
  if (m >= rows) return;
  if (PAIRED && j >= 2) return;
  const int n = n0 + j;
  if (n >= a.N) return;

  if (EPI == EPI_STORE) {
    a.Y[(size_t)map_row(a.yrow, row) * a.ldy + n] = v;
  } else if (EPI == EPI_RESID) {
    const float r = a.R[(size_t)map_row(a.rrow, row) * a.ldr + n];
    a.Y[(size_t)map_row(a.yrow, row) * a.ldy + n] = r + v;
  } else if (EPI == EPI_QKV) {
    if (n < a.nsplit)
      a.Y[(size_t)row * a.ldy + n] = v;
    else
      a.Y2[(size_t)map_row(a.y2row, row) * a.ldy2 + (n - a.nsplit)] = v;
  } else if (EPI == EPI_SILU) {
    a.Y[(size_t)map_row(a.yrow, row) * a.ldy + n] = silu(v);
  } else if (EPI == EPI_SWIGLU) {
    a.Y[(size_t)map_row(a.yrow, row) * a.ldy + n] = silu(v) * v2;
  } else if (EPI == EPI_HEAD) {
    const HeadOut& h = a.head;
    const float mu = fmaf(h.gmu[n], v, h.bmu[n]);
    const float raw = fmaf(h.gsig[n], v2, h.bsig[n]);
    const float ls = fminf(h.ln_smax, fmaxf(h.ln_smin, raw));
    const float sg = expf(ls);
    const size_t o = (size_t)map_row(a.yrow, row) * a.N + n;
    h.mean[o] = mu;
    h.scale[o] = sg;
    int32_t c;
    uint16_t x;
    select_table(mu, ls, h.ln_smin, h.inv_delta, &c, &x);
    h.center[o] = c;
    h.index[o] = x;
    if (h.center_c) {
      h.center_c[(size_t)row * a.N + n] = c;
      h.index_c[(size_t)row * a.N + n] = x;
    }
    if (!(fabsf(mu) <= FLT_MAX) || !(fabsf(raw) <= FLT_MAX)) atomicOr(h.flag, 1);
  }
}

// Kernels whose dynamic LDS can exceed 64 KiB opt in to the full 160 KiB.
inline bool allow_big_lds(const void* fn) {
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) ==
         hipSuccess;
}

template <int AK, bool RMS, int EPI>
void launch_gemm(const GemmArgs& a, hipStream_t s) {
  constexpr bool PAIRED = (EPI == EPI_SWIGLU || EPI == EPI_HEAD);
  const int K4 = a.K / 4;
  const int per_block = kWaves * (PAIRED ? 2 : kRowsW);
  dim3 grid((a.N + per_block - 1) / per_block, (a.M + kMB - 1) / kMB);
  const size_t tile = (size_t)kMB * a.K * sizeof(float);
  const size_t red = (size_t)kWaves * 64 * 65 * sizeof(float);
  const size_t lds = tile > red ? tile : red;
#define PSWA_KC(n)                                                                  \
  if (K4 <= 64 * n) {                                                               \
    static const bool attr_set = allow_big_lds(                                     \
        reinterpret_cast<const void*>(&k_gemm<AK, RMS, EPI, n>));                   \
    (void)attr_set;                                                                 \
    hipLaunchKernelGGL((k_gemm<AK, RMS, EPI, n>), grid, dim3(256), lds, s, a);      \
    return;                                                                         \
  }
  PSWA_KC(1);
  PSWA_KC(2);
  PSWA_KC(4);
  PSWA_KC(6);
  PSWA_KC(8);
#undef PSWA_KC
}

// ----------------------------------------------------------- attention
// One 64-lane wave per (query row, head). Lane l owns keys l, l+64, ... in
// slot order (spatial window, then the null slot or the temporal windows)
// and runs an online softmax over them, loading each key's K and V rows
// together. The lanes are then merged: common max by a wave reduction, the
// rescaled exp-sums by a wave reduction, and the rescaled value vectors
// summed lane 0..63 in order through LDS. All orders are fixed.
constexpr int kMaxKeys = 256;


template <int DH>
__global__ void __launch_bounds__(256) k_attn(AttnArgs a) {
  __shared__ float tr[4][DH][65];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int item = blockIdx.x * 4 + wave;
  const bool live = item < a.M * a.heads;  // no early exit: the block syncs below
  const int m = live ? item / a.heads : 0, hd = live ? item % a.heads : 0;
  const int p = map_row(a.pos, m);
  const int pi = p / a.W, pj = p % a.W;
  const int r = a.r, k1 = 2 * r + 1;
  const int n_causal = 2 * r * (r + 1);
  const int n_sp = n_causal + (a.include_self ? 1 : 0);
  const int n_tm = a.tkv ? 2 * k1 * k1 : 0;
  const int n_keys = live ? n_sp + (a.knull ? 1 : 0) + n_tm : 0;
  const int d = a.d;
  const float scale = 1.0f / sqrtf(float(DH));

  float4 q[DH / 4];
  {
    const float* qv = a.q + (size_t)m * a.ldq + hd * DH;
#pragma unroll
    for (int e = 0; e < DH / 4; ++e) q[e] = *reinterpret_cast<const float4*>(qv + 4 * e);
  }

  float mx = -INFINITY, sum = 0.f;
  float o[DH];
#pragma unroll
  for (int e = 0; e < DH; ++e) o[e] = 0.f;

#pragma unroll
  for (int u = 0; u < kMaxKeys / 64; ++u) {
    const int kk = lane + 64 * u;
    if (kk >= n_keys) continue;
    const float* kp = nullptr;
    const float* vp = nullptr;
    float b = 0.f;
    if (kk < n_sp) {
      int da, db;
      if (kk < r * k1) {
        da = kk / k1 - r;
        db = kk % k1 - r;
      } else if (kk < n_causal) {
        da = 0;
        db = kk - r * k1 - r;
      } else {
        da = 0;
        db = 0;
      }
      const int ki = pi + da, kj = pj + db;
      if (ki < 0 || ki >= a.H || kj < 0 || kj >= a.W) continue;
      kp = a.kv + (size_t)(ki * a.W + kj) * 2 * d + hd * DH;
      vp = kp + d;
      b = a.bias[hd * a.nbias + kk];
    } else if (a.knull && kk == n_sp) {
      kp = a.knull + hd * DH;
      vp = a.vnull + hd * DH;
    } else {
      const int t = kk - n_sp - (a.knull ? 1 : 0);
      const int tau = t / (k1 * k1), rem = t % (k1 * k1);
      const int ki = pi + rem / k1 - r, kj = pj + rem % k1 - r;
      if (ki < 0 || ki >= a.H || kj < 0 || kj >= a.W) continue;
      kp = a.tkv + ((size_t)tau * a.H * a.W + (size_t)(ki * a.W + kj)) * 2 * d + hd * DH;
      vp = kp + d;
      b = a.bias[hd * a.nbias + n_sp + t];
    }
    float4 kr[DH / 4], vr[DH / 4];
#pragma unroll
    for (int e = 0; e < DH / 4; ++e) {
      kr[e] = *reinterpret_cast<const float4*>(kp + 4 * e);
      vr[e] = *reinterpret_cast<const float4*>(vp + 4 * e);
    }
    float dot = 0.f;
#pragma unroll
    for (int e = 0; e < DH / 4; ++e) dot = dot4(q[e], kr[e], dot);
    const float lg = dot * scale + b;
    const float mn = fmaxf(mx, lg);
    const float c_old = expf(mx - mn);  // 0 for the first key (mx = -inf)
    const float pk = expf(lg - mn);
    sum = sum * c_old + pk;
#pragma unroll
    for (int e = 0; e < DH / 4; ++e) {
      o[4 * e + 0] = fmaf(pk, vr[e].x, o[4 * e + 0] * c_old);
      o[4 * e + 1] = fmaf(pk, vr[e].y, o[4 * e + 1] * c_old);
      o[4 * e + 2] = fmaf(pk, vr[e].z, o[4 * e + 2] * c_old);
      o[4 * e + 3] = fmaf(pk, vr[e].w, o[4 * e + 3] * c_old);
    }
    mx = mn;
  }

  const float gmx = wave_max(mx);
  const float f = mx == -INFINITY ? 0.f : expf(mx - gmx);
  const float tot = wave_sum(sum * f);
#pragma unroll
  for (int e = 0; e < DH; ++e) tr[wave][e][lane] = o[e] * f;
  __syncthreads();
  if (live && lane < DH) {
    float v = 0.f;
#pragma unroll
    for (int l = 0; l < 64; ++l) v += tr[wave][lane][l];
    a.out[(size_t)m * a.ldo + hd * DH + lane] = v / tot;
  }
}

// ---------------------------------------------------------------- misc

__global__ void k_hyper_embed(const int32_t* z, int Hh, int Wh, int Ch, const float* Wm,
                              const float* P4, int H, int W, int d, float* h) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)H * W * d) return;
  const int n = idx % d;
  const int p = idx / d;
  const int i = p / W, j = p % W;
  const int32_t* zr = z + ((size_t)(i / 4) * Wh + (j / 4)) * Ch;
  const float* wr = Wm + (size_t)n * Ch;
  float acc = 0.f;
  for (int k = 0; k < Ch; ++k) acc = fmaf(float(zr[k]), wr[k], acc);
  h[idx] = acc + P4[((i % 4) * 4 + (j % 4)) * d + n];
}

__global__ void k_gather_symbols(const int32_t* src, int compact, const int* pos, int M, int C,
                                 int32_t* ydec) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)M * C) return;
  const int m = idx / C, c = idx % C;
  const int p = map_row(pos, m);
  ydec[(size_t)p * C + c] = src[(size_t)(compact ? m : p) * C + c];
}

__global__ void k_symbol_bits(const int* pos, int M, int C, const int32_t* ydec,
                              const float* mean, const float* scale, float* bits) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)M * C) return;
  const int m = idx / C, c = idx % C;
  const size_t o = (size_t)map_row(pos, m) * C + c;
  const float v = fabsf(float(ydec[o]) - mean[o]);
  const float s2 = scale[o] * 1.41421356237309515f;
  const float p = 0.5f * (erfcf((v - 0.5f) / s2) - erfcf((v + 0.5f) / s2));
  bits[o] = -log2f(fmaxf(p, 1e-9f));
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
// a step. Position (i, j) lands at start(t) + (i - i_lo(t)).
__global__ void k_fill_positions(int H, int W, int s, int* pos_all) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= H * W) return;
  const int i = p / W, j = p % W;
  const int t = j + s * i;
  // start(t) = number of positions with step < t = sum over rows i' of
  // clamp(t - s*i', 0, W).
  long start = 0;
  for (int ii = 0; ii < H; ++ii) start += min(max(t - s * ii, 0), W);
  const int i_lo = max(0, (t - W + s) / s);  // smallest i with t - s*i <= W-1
  pos_all[start + (i - i_lo)] = p;
}

inline unsigned blocks_for(long n, int t) { return unsigned((n + t - 1) / t); }

}  // namespace

void gemm_f32(AKind ak, bool rms, Epi epi, const GemmArgs& a, hipStream_t s) {
  if (a.M <= 0) return;
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
}

void attention_f32(const AttnArgs& a, hipStream_t s) {
  if (a.M <= 0) return;
  const dim3 grid(blocks_for((long)a.M * a.heads, 4));
  switch (a.dh) {  // other head sizes are rejected when the model is created
    case 16: hipLaunchKernelGGL(k_attn<16>, grid, dim3(256), 0, s, a); break;
    case 32: hipLaunchKernelGGL(k_attn<32>, grid, dim3(256), 0, s, a); break;
    case 48: hipLaunchKernelGGL(k_attn<48>, grid, dim3(256), 0, s, a); break;
    case 64: hipLaunchKernelGGL(k_attn<64>, grid, dim3(256), 0, s, a); break;
    default: break;
  }
}

void hyper_embed(const int32_t* z, int Hh, int Wh, int Ch, const float* Wm, const float* P4,
                 int H, int W, int d, float* h, hipStream_t s) {
  hipLaunchKernelGGL(k_hyper_embed, dim3(blocks_for((long)H * W * d, 256)), dim3(256), 0, s, z,
                     Hh, Wh, Ch, Wm, P4, H, W, d, h);
}

void gather_symbols(const int32_t* src, int compact, const int* pos, int M, int C,
                    int32_t* ydec, hipStream_t s) {
  if (M <= 0) return;
  hipLaunchKernelGGL(k_gather_symbols, dim3(blocks_for((long)M * C, 256)), dim3(256), 0, s, src,
                     compact, pos, M, C, ydec);
}

void symbol_bits(const int* pos, int M, int C, const int32_t* ydec, const float* mean,
                 const float* scale, float* bits, hipStream_t s) {
  if (M <= 0) return;
  hipLaunchKernelGGL(k_symbol_bits, dim3(blocks_for((long)M * C, 256)), dim3(256), 0, s, pos, M,
                     C, ydec, mean, scale, bits);
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

void fill_positions(int H, int W, int s, int* pos_all, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_positions, dim3(blocks_for((long)H * W, 256)), dim3(256), 0, st, H,
                     W, s, pos_all);
}

}  // namespace pswa
