// Device building blocks shared by the per-launch kernels (kernels_f32.hip)
// and the persistent decode kernel (persistent.hip). Every output is computed
// by the same code whatever launch runs it, and the library is built with
// -ffp-contract=off, so a row's values are bit-identical across the parallel
// encode form, the per-diagonal decode and the persistent multi-frame decode.
#pragma once

#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

#include "pswa_internal.h"

namespace pswa {
namespace dev {

constexpr float kEps = 1e-5f;
constexpr int kRowsW = 4;   // weight rows per wave in a GEMM tile
constexpr int kWaves = 4;   // waves per 256-thread block
constexpr int kMB = 16;     // A rows per GEMM tile
constexpr int kMaxKeys = 256;
constexpr int kThreads = 256;

// Global-memory accesses through generic pointers. Pointers that device code
// reads from argument tables in device memory are generic, and generic
// (flat) accesses also count against the LDS wait counter, so every block
// barrier and every LDS wait would also wait for them. These accessors
// address global memory directly (HIP's float4 / int4 go through native
// vectors: a class type in another address space is copied with flat
// accesses).
template <typename T> using gptr = __attribute__((address_space(1))) T*;
typedef float f32x4v __attribute__((ext_vector_type(4)));
typedef int i32x4v __attribute__((ext_vector_type(4)));
template <typename T>
__device__ __forceinline__ T ldg(const T* p) {
  return *(gptr<const T>)p;
}
__device__ __forceinline__ float4 ldg(const float4* p) {
  const f32x4v v = *(gptr<const f32x4v>)(const void*)p;
  return make_float4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ int4 ldg(const int4* p) {
  const i32x4v v = *(gptr<const i32x4v>)(const void*)p;
  return make_int4(v[0], v[1], v[2], v[3]);
}
template <typename T>
__device__ __forceinline__ void stg(T* p, T v) {
  *(gptr<T>)p = v;
}
__device__ __forceinline__ float4 ldg4(const float* p) {
  return ldg(reinterpret_cast<const float4*>(p));
}

// FP32 -> BF16, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
// Two BF16 values packed in a word (element 2j in the low half) -> floats.
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }
__device__ __forceinline__ int4 ldg4(const int32_t* p) {
  return ldg(reinterpret_cast<const int4*>(p));
}

// A struct from a read-only table in device memory at a wave-uniform address,
// read with scalar loads into registers (the table is never written while a
// kernel runs).
template <typename S>
__device__ __forceinline__ S load_uniform(const S* p) {
  static_assert(sizeof(S) % 4 == 0, "table entries are whole words");
  constexpr int kWords = sizeof(S) / 4;
  typedef __attribute__((address_space(4))) const int* cptr;
  const cptr src = (cptr)(const void*)p;
  int w[kWords];
#pragma unroll
  for (int i = 0; i < kWords; ++i) w[i] = src[i];
  S out;
  __builtin_memcpy(&out, w, sizeof(S));
  return out;
}

// A struct that every lane reads at the same LDS address, moved into scalar
// registers.
template <typename S>
__device__ __forceinline__ S lds_uniform(const S* p) {
  static_assert(sizeof(S) % 4 == 0, "table entries are whole words");
  constexpr int kWords = sizeof(S) / 4;
  const int* src = reinterpret_cast<const int*>(p);
  int w[kWords];
#pragma unroll
  for (int i = 0; i < kWords; ++i) w[i] = __builtin_amdgcn_readfirstlane(src[i]);
  S out;
  __builtin_memcpy(&out, w, sizeof(S));
  return out;
}

// Block-wide copy of n words from device memory to LDS, 16 loads per thread
// in flight per round (ends without a block barrier).
__device__ __forceinline__ void copy_words_to_lds(int* dst, const int* src, int n) {
  for (int base = 0; base < n; base += 16 * kThreads) {
    int v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int i = min(base + u * kThreads + (int)threadIdx.x, n - 1);
      v[u] = ldg(src + i);
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int i = base + u * kThreads + (int)threadIdx.x;
      if (i < n) dst[i] = v[u];
    }
  }
}

__device__ __forceinline__ int map_row(const int* idx, int m) { return idx ? ldg(idx + m) : m; }

__device__ __forceinline__ float silu(float v) { return v / (1.0f + expf(-v)); }

__device__ __forceinline__ float dot4(float4 x, float4 w, float acc) {
  acc = fmaf(x.x, w.x, acc);
  acc = fmaf(x.y, w.y, acc);
  acc = fmaf(x.z, w.z, acc);
  return fmaf(x.w, w.w, acc);
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

// RMSNorm of one row's K-value slice x (wave per row): lane l sums x[k]^2
// for k = l, l + 64, ... with fmaf in order, then a fixed xor tree;
// y[k] = x[k] * rs * gain[k].
__device__ __forceinline__ void group_rms_row(const float* x, const float* gain, float* y, int K) {
  const int lane = threadIdx.x & 63;
  float ss = 0.f;
  for (int k = lane; k < K; k += 64) {
    const float v = ldg(x + k);
    ss = fmaf(v, v, ss);
  }
  ss = wave_sum(ss);
  const float rs = 1.0f / sqrtf(ss / float(K) + kEps);
  for (int k = lane; k < K; k += 64) stg(y + k, ldg(x + k) * rs * ldg(gain + k));
}

// Centre and table index of one symbol, one rounding per operation, so the
// decision equals the documented float32 formula.
__device__ __forceinline__ void select_table(float mu, float lsig, float ln_smin, float inv_delta,
                                             int32_t* c_out, uint16_t* i_out) {
  const float c = floorf(mu + 0.5f);
  const float ph = (mu - c) + 0.5f;
  const float m = fminf(15.0f, floorf(ph * 16.0f));
  const float t = (lsig - ln_smin) * inv_delta;
  const float s = fminf(63.0f, fmaxf(0.0f, floorf(t + 0.5f)));
  *c_out = int32_t(c);
  *i_out = uint16_t(int(s) * 16 + int(m));
}

// Number of float4 chunks per lane a GEMM with reduction length K needs
// (a compile-time count per instantiation; chunks past K are skipped).
__host__ __device__ inline int kc_for(int K) {
  const int K4 = K / 4;
  return K4 <= 64 ? 1 : K4 <= 128 ? 2 : K4 <= 256 ? 4 : 8;
}

__host__ __device__ inline constexpr bool paired_epi(int epi) {
  return epi == EPI_SWIGLU || epi == EPI_HEAD;
}

// Tiles of a GEMM launch: (column tiles, row tiles).
__host__ __device__ inline int gemm_col_tiles(int N, int epi) {
  const int per = kWaves * (paired_epi(epi) ? 2 : kRowsW);
  return (N + per - 1) / per;
}
__host__ __device__ inline int gemm_row_tiles(int M) { return (M + kMB - 1) / kMB; }

// LDS a GEMM tile needs: the raw A tile, reused as the lane-transpose buffer.
__host__ __device__ inline size_t gemm_lds_bytes(int K) {
  const size_t tile = (size_t)kMB * K * sizeof(float);
  const size_t red = (size_t)kWaves * 64 * 65 * sizeof(float);
  return tile > red ? tile : red;
}

// -log2(max(P, 1e-9)) of integer symbol y under the discretised Gaussian
// N(mean, scale): P = Phi((|y - mean| + 1/2) / scale) - Phi((|y - mean| - 1/2) / scale),
// written with erfc.
__device__ __forceinline__ float symbol_bits_of(int32_t y, float mean, float scale) {
  const float v = fabsf(float(y) - mean);
  const float s2 = scale * 1.41421356237309515f;
  const float p = 0.5f * (erfcf((v - 0.5f) / s2) - erfcf((v + 0.5f) / s2));
  return -log2f(fmaxf(p, 1e-9f));
}

// Epilogue of one GEMM output (row, n): v is the finished dot product with
// W, v2 the one with W2 (paired epilogues only).
template <int EPI>
__device__ __forceinline__ void epilogue(const GemmArgs& a, int row, int n, float v, float v2) {
  if (EPI == EPI_STORE) {
    const size_t o = (size_t)map_row(a.yrow, row) * a.ldy + n;
    if (a.kv16) stg(reinterpret_cast<uint16_t*>(a.Y) + o, bf16_rne(v));
    else stg(a.Y + o, v);
  } else if (EPI == EPI_RESID) {
    const float r = ldg(a.R + (size_t)map_row(a.rrow, row) * a.ldr + n);
    stg(a.Y + (size_t)map_row(a.yrow, row) * a.ldy + n, r + v);
  } else if (EPI == EPI_QKV) {
    if (n < a.nsplit) {
      stg(a.Y + (size_t)row * a.ldy + n, v);
    } else {
      const size_t o = (size_t)map_row(a.y2row, row) * a.ldy2 + (n - a.nsplit);
      if (a.kv16) stg(reinterpret_cast<uint16_t*>(a.Y2) + o, bf16_rne(v));
      else stg(a.Y2 + o, v);
    }
  } else if (EPI == EPI_SILU) {
    stg(a.Y + (size_t)map_row(a.yrow, row) * a.ldy + n, silu(v));
  } else if (EPI == EPI_SWIGLU) {
    stg(a.Y + (size_t)map_row(a.yrow, row) * a.ldy + n, silu(v) * v2);
  } else if (EPI == EPI_HEAD) {
    const HeadOut& h = a.head;
    const int cn = h.col0 + n;  // the output channel
    const float mu = fmaf(ldg(h.gmu + cn), v, ldg(h.bmu + cn));
    const float raw = fmaf(ldg(h.gsig + cn), v2, ldg(h.bsig + cn));
    const float ls = fminf(h.ln_smax, fmaxf(h.ln_smin, raw));
    const float sg = expf(ls);
    const size_t o = (size_t)map_row(a.yrow, row) * h.ldo + cn;
    stg(h.mean + o, mu);
    stg(h.scale + o, sg);
    int32_t c;
    uint16_t x;
    select_table(mu, ls, h.ln_smin, h.inv_delta, &c, &x);
    stg(h.center + o, c);
    stg(h.index + o, x);
    if (h.center_c) {
      stg(h.center_c + (size_t)row * h.ldo + cn, c);
      stg(h.index_c + (size_t)row * h.ldo + cn, x);
    }
    if (h.ydec) {  // the row's symbol and its bits, from the values just computed
      const int32_t y = ldg(h.ysrc + (h.src_compact ? (size_t)row * h.ldo + cn : o));
      stg(h.ydec + o, y);
      stg(h.bits + o, symbol_bits_of(y, mu, sg));
    }
    if (!(fabsf(mu) <= FLT_MAX) || !(fabsf(raw) <= FLT_MAX)) atomicOr(h.flag, 1);
  }
}

// ---------------------------------------------------------------- GEMM tile
// Skinny FP32 GEMM tile: 16 weight rows (4 per wave) x up to 16 A rows.
//   1. each wave loads its 4 weight rows into registers: lane l takes the
//      float4 chunks l, l + 64, ... (KC of them, all in flight);
//   2. the block stages the raw A tile [rows][K] in LDS, 8 loads per thread
//      in flight;
//   3. RMSNorm rows: lane l sums x^2 over its chunks in order, then a fixed
//      xor tree gives the row's 1/rms;
//   4. each lane keeps an fmaf chain per (row, weight row) over its chunks,
//      and the 64 lane partials are summed lane 0..63 in order.
// The RMSNorm scale is applied to the finished dot product:
//   sum_k (x_k * rstd * g_k) w_k  ==  rstd * sum_k (x_k g_k) w_k.
// An output's arithmetic depends only on K. Paired epilogues (SwiGLU, head):
// a wave's weight rows are W[n], W[n+1], W2[n], W2[n+1] -> outputs n, n+1.
template <int AK, bool RMS, int EPI, int KC>
__device__ __forceinline__ void gemm_tile(const GemmArgs& a, int bx, int by, float4* smem4, float* rstd) {
  constexpr bool PAIRED = paired_epi(EPI);
  float* smem = reinterpret_cast<float*>(smem4);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n0 = bx * kWaves * (PAIRED ? 2 : kRowsW) + wave * (PAIRED ? 2 : kRowsW);
  const int m0 = by * kMB;
  const int K = a.K, K4 = a.K / 4;
  const int rows = min(kMB, a.M - m0);
  __syncthreads();  // the previous tile of this block is done with the LDS

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
      w[it][j] = in ? ldg4(wrow[j] + 4 * c) : make_float4(0, 0, 0, 0);
    g[it] = make_float4(1.f, 1.f, 1.f, 1.f);
    if (RMS && in) g[it] = ldg4(a.gain + 4 * c);
    if (AK == A_INT && in) g[it] = ldg4(a.xscale + 4 * c);
  }

  {
    const int total = rows * K4;
    for (int base = 0; base < total; base += 8 * kThreads) {
      float4 x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = base + u * kThreads + tid;
        x[u] = make_float4(0.f, 0.f, 0.f, 0.f);  // (keeps x in registers)
        if (e < total) {
          const int m = e / K4, c = e % K4;
          const size_t off = (size_t)map_row(a.xrow, m0 + m) * a.ldx + 4 * c;
          if (AK == A_INT) {
            const int4 xi = ldg4(a.Xi + off);
            x[u] = make_float4(float(xi.x), float(xi.y), float(xi.z), float(xi.w));
          } else {
            x[u] = ldg4(a.X + off);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = base + u * kThreads + tid;
        if (e < total) smem4[e] = x[u];
      }
    }
  }
  __syncthreads();

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
  if (a.amax) {
    // calibration: the largest |value| this projection multiplies (the
    // RMSNorm output, or the input times its scale), over the tile's rows
    float mx = 0.f;
    for (int m = wave; m < rows; m += kWaves) {
      float rm = 0.f, ss = 0.f;
#pragma unroll
      for (int it = 0; it < KC; ++it) {
        const int c = lane + 64 * it;
        if (c < K4) {
          const float4 x = smem4[m * K4 + c];
          if (RMS) ss = dot4(x, x, ss);
          rm = fmaxf(rm, fmaxf(fmaxf(fabsf(x.x * g[it].x), fabsf(x.y * g[it].y)),
                               fmaxf(fabsf(x.z * g[it].z), fabsf(x.w * g[it].w))));
        }
      }
      rm = wave_max(rm);
      if (RMS) rm *= 1.0f / sqrtf(wave_sum(ss) / float(K) + kEps);
      mx = fmaxf(mx, rm);
    }
    // non-negative floats order as their bit patterns
    if (lane == 0 && mx > 0.f) atomicMax(reinterpret_cast<unsigned*>(a.amax), __float_as_uint(mx));
  }

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

  epilogue<EPI>(a, row, n, v, v2);
}

// Runtime choice of the chunk count (the same choice everywhere).
template <int AK, bool RMS, int EPI>
__device__ __forceinline__ void gemm_tile_any(const GemmArgs& a, int bx, int by, float4* smem4,
                                              float* rstd) {
  switch (kc_for(a.K)) {
    case 1: gemm_tile<AK, RMS, EPI, 1>(a, bx, by, smem4, rstd); break;
    case 2: gemm_tile<AK, RMS, EPI, 2>(a, bx, by, smem4, rstd); break;
    case 4: gemm_tile<AK, RMS, EPI, 4>(a, bx, by, smem4, rstd); break;
    default: gemm_tile<AK, RMS, EPI, 8>(a, bx, by, smem4, rstd); break;
  }
}

// ------------------------------------------------------------ attention item
// Sum of a LEN-element vector over the lanes of a wave, scattered: while the
// length is even and lane-distance masks remain, partners (lane ^ MASK)
// exchange halves and each keeps the sum of one half (the lane with the mask
// bit set keeps the upper half, and off grows by LEN / 2 for it); the odd
// remainder is then summed over the remaining masks in every lane of a group
// of `group` lanes. Each sum adds the same two operands in both partners, so
// every lane that holds an element holds the same bits, and the tree is the
// same in every launch. On return v[0 .. merge_len) holds elements off ..
// off + merge_len - 1 of the total.
template <int LEN, int MASK>
__host__ __device__ constexpr int merge_len() {
  if constexpr (MASK > 0 && LEN % 2 == 0) return merge_len<LEN / 2, MASK / 2>();
  else return LEN;
}
template <int LEN, int MASK>
__device__ __forceinline__ void merge_lanes(float* v, int lane, int& off, int& group) {
  if constexpr (MASK > 0 && LEN % 2 == 0) {
    constexpr int H = LEN / 2;
    const bool upper = (lane & MASK) != 0;
    // in place: step j reads only v[j] and v[H + j]
#pragma unroll
    for (int j = 0; j < H; ++j) {
      const float send = upper ? v[j] : v[H + j];
      const float keep = upper ? v[H + j] : v[j];
      v[j] = keep + __shfl_xor(send, MASK, 64);
    }
    if (upper) off += H;
    merge_lanes<H, MASK / 2>(v, lane, off, group);
  } else {
#pragma unroll
    for (int mk = MASK; mk > 0; mk >>= 1) {
#pragma unroll
      for (int j = 0; j < LEN; ++j) v[j] = v[j] + __shfl_xor(v[j], mk, 64);
    }
    group = 2 * MASK > 0 ? 2 * MASK : 1;
  }
}

// Attention items: one 64-lane wave per (query row, pair of heads); lanes
// 0-31 compute head 2p and lanes 32-63 head 2p + 1 (idle when the head count
// is odd and 2p + 1 is past it). In its half, lane l owns the key slots
// l, l + 32, ... (spatial window, then the null slot or the temporal
// windows) and runs an online softmax over them, in slot order. The K and V
// rows of NK of a lane's slots are requested together before any is used
// (NK = 2 for BF16 caches, 1 for FP32 ones), so one round trip to memory
// serves two slots. The half's lanes are then merged: common maximum and
// rescaled exp-sum by reductions over the half, the rescaled value vectors
// by the butterfly of merge_lanes (a fixed tree, in registers). Waves work
// independently (no block synchronisation and no LDS).
// Key positions: a row's frame (fid, else the single frame0) gives its grid
// and its offset in the global position space; temporal K/V of frame
// position g in previous frame tau is at (tau * HWt + g) * 2d; the
// accumulator's null key and value are the row after the last position
// (HWt) of its cache.
constexpr int kHalf = 32;

__device__ __forceinline__ float half_max(float v) {
#pragma unroll
  for (int o = kHalf / 2; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ float half_sum(float v) {
#pragma unroll
  for (int o = kHalf / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
// lanes sharing each merged element at the end of merge_lanes<LEN, MASK>
template <int LEN, int MASK>
__host__ __device__ constexpr int merge_group() {
  if constexpr (MASK > 0 && LEN % 2 == 0) return merge_group<LEN / 2, MASK / 2>();
  else return 2 * MASK > 0 ? 2 * MASK : 1;
}

// The frame of query row m.
__device__ __forceinline__ FrameInfo attn_frame(const AttnArgs& a, int m) {
  if (!a.fid) return a.frame0;
  const int f = ldg(a.fid + m);
  return FrameInfo{ldg(&a.frames[f].H), ldg(&a.frames[f].W), ldg(&a.frames[f].off),
                   ldg(&a.frames[f].n_prev)};
}

// Raw K and V rows of one key slot as loaded (BF16 pairs, or FP32 bit
// patterns) and its bias: the loads are in flight until kv_widen reads them.
template <int DH>
struct KeyRaw {
  int4 k[DH / 4], v[DH / 4];  // BF16 rows use the first DH / 8 of each
  float b;
};
template <int DH, bool KV16>
__device__ __forceinline__ void kv_issue(const float* base, size_t e, int d, KeyRaw<DH>& r) {
  if constexpr (KV16) {
    const uint16_t* p = reinterpret_cast<const uint16_t*>(base) + e;
#pragma unroll
    for (int c = 0; c < DH / 8; ++c) {
      r.k[c] = ldg(reinterpret_cast<const int4*>(p) + c);
      r.v[c] = ldg(reinterpret_cast<const int4*>(p + d) + c);
    }
  } else {
#pragma unroll
    for (int c = 0; c < DH / 4; ++c) {
      r.k[c] = ldg(reinterpret_cast<const int4*>(base + e) + c);
      r.v[c] = ldg(reinterpret_cast<const int4*>(base + e + d) + c);
    }
  }
}
template <int DH, bool KV16>
__device__ __forceinline__ void kv_widen(const KeyRaw<DH>& r, float4* kr, float4* vr) {
  if constexpr (KV16) {
#pragma unroll
    for (int c = 0; c < DH / 8; ++c) {
      const int4 k8 = r.k[c], v8 = r.v[c];
      kr[2 * c] = make_float4(bf16_lo(k8.x), bf16_hi(k8.x), bf16_lo(k8.y), bf16_hi(k8.y));
      kr[2 * c + 1] = make_float4(bf16_lo(k8.z), bf16_hi(k8.z), bf16_lo(k8.w), bf16_hi(k8.w));
      vr[2 * c] = make_float4(bf16_lo(v8.x), bf16_hi(v8.x), bf16_lo(v8.y), bf16_hi(v8.y));
      vr[2 * c + 1] = make_float4(bf16_lo(v8.z), bf16_hi(v8.z), bf16_lo(v8.w), bf16_hi(v8.w));
    }
  } else {
#pragma unroll
    for (int c = 0; c < DH / 4; ++c) {
      kr[c] = make_float4(__int_as_float(r.k[c].x), __int_as_float(r.k[c].y),
                          __int_as_float(r.k[c].z), __int_as_float(r.k[c].w));
      vr[c] = make_float4(__int_as_float(r.v[c].x), __int_as_float(r.v[c].y),
                          __int_as_float(r.v[c].z), __int_as_float(r.v[c].w));
    }
  }
}

// The arithmetic of one attention item, shared by every path.
// src.issue(kk, want, slot) requests key slot kk (false: not wanted, masked
// or outside the frame; the slot then holds harmless data that is never
// used) and src.get(slot, kr, vr, b) delivers its K and V rows and bias; q4
// is the lane's head's query, out its output row. live = false idles the
// half. Every requested slot goes through the same straight-line update and
// an unused one leaves the lane's state as it was by selection, so no load
// or update sits behind a per-lane branch (the compiler's wait counters
// then keep all NK slots' loads in flight together).
template <int DH, int NK, class Source>
__device__ __forceinline__ void attn_core(const float4* q4, int n_keys, bool live, Source& src,
                                          float* out) {
  const int lane = threadIdx.x & 63, l32 = lane & (kHalf - 1);
  const float scale = 1.0f / sqrtf(float(DH));
  float mx = -INFINITY, sum = 0.f;
  float o[DH];
#pragma unroll
  for (int e = 0; e < DH; ++e) o[e] = 0.f;

#pragma unroll 1
  for (int u = 0; u < kMaxKeys / kHalf; u += NK) {
    if (kHalf * u >= n_keys) break;  // the same for the whole wave
    typename Source::Slot sl[NK];
    bool ok[NK];
#pragma unroll
    for (int j = 0; j < NK; ++j) {
      const int kk = l32 + kHalf * (u + j);
      ok[j] = src.issue(kk, live && kk < n_keys, sl[j]);
    }
    // every slot's loads are issued before the first is used
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < NK; ++j) {
      const bool use = ok[j];
      float4 kr[DH / 4], vr[DH / 4];
      float b;
      src.get(sl[j], kr, vr, b);
      float dot = 0.f;
#pragma unroll
      for (int e = 0; e < DH / 4; ++e) dot = dot4(q4[e], kr[e], dot);
      const float lg = dot * scale + b;
      const float mn = fmaxf(mx, lg);
      const float c_old = expf(mx - mn);  // 0 for the lane's first key (mx = -inf)
      const float pk = expf(lg - mn);
      sum = use ? sum * c_old + pk : sum;
#pragma unroll
      for (int e = 0; e < DH / 4; ++e) {
        o[4 * e + 0] = use ? fmaf(pk, vr[e].x, o[4 * e + 0] * c_old) : o[4 * e + 0];
        o[4 * e + 1] = use ? fmaf(pk, vr[e].y, o[4 * e + 1] * c_old) : o[4 * e + 1];
        o[4 * e + 2] = use ? fmaf(pk, vr[e].z, o[4 * e + 2] * c_old) : o[4 * e + 2];
        o[4 * e + 3] = use ? fmaf(pk, vr[e].w, o[4 * e + 3] * c_old) : o[4 * e + 3];
      }
      mx = use ? mn : mx;
    }
  }

  const float gmx = half_max(mx);
  const float f = mx == -INFINITY ? 0.f : expf(mx - gmx);
  const float tot = half_sum(sum * f);
  // lanes' rescaled value vectors summed over the half by a fixed butterfly
  float v[DH];
#pragma unroll
  for (int e = 0; e < DH; ++e) v[e] = o[e] * f;
  int off = 0, group = 1;
  merge_lanes<DH, kHalf / 2>(v, lane, off, group);
  constexpr int ML = merge_len<DH, kHalf / 2>(), MG = merge_group<DH, kHalf / 2>();
  const int k = lane & (MG - 1);
  if (!live) return;
#pragma unroll
  for (int j = 0; j < ML; ++j)  // element j of the group's run, by constant index
    if (j % MG == k) stg(out + off + j, v[j] / tot);
}

// Spatial window slot kk of a query at (pi, pj): its offset (da, db) (the
// cyclic schedule's full window in raster order; else the r rows above in
// full, the r cells to the left, then the query itself).
__device__ __forceinline__ void window_offset(const AttnArgs& a, int kk, int& da, int& db) {
  const int r = a.r, k1 = 2 * r + 1;
  if (a.cycle || kk < r * k1) {
    da = kk / k1 - r;
    db = kk % k1 - r;
  } else if (kk < 2 * r * (r + 1)) {
    da = 0;
    db = kk - r * k1 - r;
  } else {
    da = 0;
    db = 0;
  }
}

// Spatial slots of a row (with self for layers).
__device__ __forceinline__ int attn_n_sp(const AttnArgs& a) {
  const int k1 = 2 * a.r + 1;
  return a.cycle ? k1 * k1 : 2 * a.r * (a.r + 1) + (a.include_self ? 1 : 0);
}

// Where key slot kk of the query at (pi, pj) lives: the cache (temporal:
// tkv, else kv) and element offset of its K row for head hd, and its bias
// index (-1: no bias, the null slot); false when the slot is masked or
// outside the frame.
struct SlotAddr {
  bool temporal;
  size_t e;
  int bias;
};
// The two caches of an item: kv, and tkv as a byte distance from it, both in
// scalar registers. The per-lane choice of cache is then an add of 0 or the
// distance; a choice between two pointer fields becomes a choice between
// their addresses, which keeps the fields in scratch memory, and the wait
// for that scratch load serialises the key loads in flight.
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}
struct KvBases {
  uint64_t kv, dt;
  __device__ __forceinline__ const float* of(const SlotAddr& s) const {
    const uint64_t add = s.temporal ? dt : 0;
    return reinterpret_cast<const float*>(kv + add);
  }
};
__device__ __forceinline__ KvBases kv_bases(const AttnArgs& a) {
  const uint64_t kv = reinterpret_cast<uint64_t>(a.kv);
  const uint64_t dt = a.tkv ? reinterpret_cast<uint64_t>(a.tkv) - kv : 0;
  return KvBases{uniform_u64(kv), uniform_u64(dt)};
}
__device__ __forceinline__ bool slot_addr(const AttnArgs& a, int kk, int hd, int dh, int pi,
                                          int pj, const FrameInfo& fi, int n_sp, int step_p,
                                          SlotAddr& s) {
  const int d = a.d;
  if (kk < n_sp) {
    int da, db;
    window_offset(a, kk, da, db);
    const int ki = pi + da, kj = pj + db;
    if (ki < 0 || ki >= fi.H || kj < 0 || kj >= fi.W) return false;
    if (a.cycle) {  // decoded early enough: strictly (accumulator) or not
      const int step_k = (ki + kj) % a.cycle;
      if (a.include_self ? step_k > step_p : step_k >= step_p) return false;
    }
    s = SlotAddr{false, (size_t)(fi.off + ki * fi.W + kj) * 2 * d + hd * dh, hd * a.nbias + kk};
    return true;
  }
  if (a.knull && kk == n_sp) {
    s = SlotAddr{false, (size_t)a.HWt * 2 * d + hd * dh, -1};
    return true;
  }
  const int r = a.r, k1 = 2 * r + 1;
  const int t = kk - n_sp - (a.knull ? 1 : 0);
  const int tau = t / (k1 * k1), rem = t % (k1 * k1);
  const int ki = pi + rem / k1 - r, kj = pj + rem % k1 - r;
  if (ki < 0 || ki >= fi.H || kj < 0 || kj >= fi.W) return false;
  s = SlotAddr{true, ((size_t)tau * a.HWt + (size_t)(fi.off + ki * fi.W + kj)) * 2 * d + hd * dh,
               hd * a.nbias + n_sp + t};
  return true;
}

// Key slots of a query row: spatial window (with self for layers), the null
// slot, the temporal windows of P-frames.
__device__ __forceinline__ int attn_n_keys(const AttnArgs& a, const FrameInfo& fi) {
  const int k1 = 2 * a.r + 1;
  return attn_n_sp(a) + (a.knull ? 1 : 0) + (a.tkv && fi.n_prev > 0 ? 2 * k1 * k1 : 0);
}

// Keys read from the caches in global memory.
template <int DH, bool KV16>
struct GlobalKeys {
  struct Slot {
    KeyRaw<DH> raw;
    bool no_bias;  // the null slot: bias 0 (chosen when the slot is used)
  };
  const AttnArgs& a;
  KvBases kb;
  int hd, pi, pj, n_sp, step_p;
  FrameInfo fi;
  __device__ __forceinline__ bool issue(int kk, bool want, Slot& sl) {
    SlotAddr s;
    const bool ok = want && slot_addr(a, kk, hd, DH, pi, pj, fi, n_sp, step_p, s);
    if (!ok) s = SlotAddr{false, 0, 0};  // unused: the first row of kv
    sl.no_bias = s.bias < 0;
    sl.raw.b = ldg(a.bias + (s.bias >= 0 ? s.bias : 0));
    kv_issue<DH, KV16>(kb.of(s), s.e, a.d, sl.raw);
    return ok;
  }
  __device__ __forceinline__ void get(const Slot& sl, float4* kr, float4* vr, float& b) {
    kv_widen<DH, KV16>(sl.raw, kr, vr);
    b = sl.no_bias ? 0.f : sl.raw.b;
  }
};

// Item (row m, head pair p) with the row's global position gp, frame fi and
// query row qr already known, every key from global memory.
template <int DH, bool KV16>
__device__ __forceinline__ void attn_pair_at(const AttnArgs& a, int m, int p, int gp,
                                             const FrameInfo& fi, int qr) {
  const int hd = 2 * p + ((threadIdx.x >> 5) & 1);
  const bool live = hd < a.heads;
  const int lp = gp - fi.off;
  const int pi = lp / fi.W, pj = lp % fi.W;
  const int n_sp = attn_n_sp(a);
  const float* qp = a.q + (size_t)qr * a.ldq + min(hd, a.heads - 1) * DH;
  float4 q4[DH / 4];
#pragma unroll
  for (int e = 0; e < DH / 4; ++e) q4[e] = ldg4(qp + 4 * e);
  GlobalKeys<DH, KV16> src{a, kv_bases(a), hd, pi, pj, n_sp, a.cycle ? (pi + pj) % a.cycle : 0, fi};
  attn_core<DH, KV16 ? 2 : 1>(q4, attn_n_keys(a, fi), live, src,
                              a.out + (size_t)m * a.ldo + hd * DH);
}

// Head pairs of a row.
__host__ __device__ inline int attn_pairs(int heads) { return (heads + 1) / 2; }

// Per-launch item `item` = m * pairs + p (rows past M idle).
template <int DH, bool KV16>
__device__ __forceinline__ void attn_item(const AttnArgs& a, int item) {
  const int np = attn_pairs(a.heads);
  if (item >= a.M * np) return;
  const int m = item / np, p = item % np;
  attn_pair_at<DH, KV16>(a, m, p, map_row(a.pos, m), attn_frame(a, m), map_row(a.qrow, m));
}

// Attention needs no LDS (the lanes are merged in registers).
__host__ __device__ inline size_t attn_lds_bytes(int) { return 0; }

// ------------------------------------------------ LDS-staged window tiles
// Attention of the persistent wavefront decode: a block takes up to
// kStageRows consecutive diagonal rows of one frame (query rows i0 .. i1 =
// i0 + R - 1 at columns j(i) = j0 - s (i - i0)) and stages the union of
// their causal windows in LDS, stage_heads heads at a time, with direct
// global-to-LDS loads: per window cell an 896-byte slot holding the K and V
// rows of those heads (one wave's load per cell), then the rows' queries and
// the heads' window biases.
// Each wave then computes its row's items for those heads from LDS alone
// (for P-frames the temporal keys come from global memory). In image row ii
// (i0 - r .. i1) the union is the column range [j(hi) - r, j(lo) + r] of the
// query rows lo .. hi whose windows hold ii (windows of neighbouring
// diagonal rows overlap, s <= 2r + 1), clipped to the frame; cells are
// numbered image row by image row, and the accumulator's null key and value
// (the row after the last position of its cache) follow as one more cell. A
// cell's data starts 16 (cell mod 8) bytes into its slot, so that lanes
// reading different cells spread over the banks. BF16 caches (kv16) are
// staged as they are, twice as many heads per slot, and widened on reading.
constexpr int kStageRows = kWaves;             // query rows of a tile (one per wave)
constexpr int kStageImgRows = kStageRows + 4;  // image rows of a tile (r <= 4)
constexpr int kStageCells = 133;               // window cells (at most 132: r = 4, s = 5) + null
constexpr int kStageCellBytes = 896;           // 56 16-byte slots per cell
// heads staged together: their K and V rows fill at most 48 of a cell's 56
// 16-byte slots (the rest is room for the skew of up to 7 slots)
__host__ __device__ inline constexpr int stage_heads(int dh, bool kv16 = false) {
  return (96 / dh > 0 ? 96 / dh : 1) * (kv16 ? 2 : 1);
}
// byte offsets of the queries and the biases after the cells
constexpr size_t kStageQOff = (size_t)kStageCells * kStageCellBytes;
__host__ __device__ inline constexpr size_t stage_bias_off(int dh, bool kv16 = false) {
  return kStageQOff + (size_t)kStageRows * stage_heads(dh, kv16) * dh * 4;
}
__host__ __device__ inline size_t attn_stage_lds_bytes(int dh, bool kv16 = false) {
  return stage_bias_off(dh, kv16) + (size_t)stage_heads(dh, kv16) * 64 * 4;
}

// ------------------------------------------------------------ symbol items
// ydec[pos(m)][c0 + c] = src[(compact ? m : pos(m))][c0 + c], idx = m * nc + c
__device__ __forceinline__ void gather_item(const int32_t* src, int compact, const int* pos, int C,
                                            int32_t* ydec, long idx, int c0 = 0, int nc = -1) {
  if (nc < 0) nc = C;
  const int m = idx / nc, c = c0 + idx % nc;
  const int p = map_row(pos, m);
  stg(ydec + (size_t)p * C + c, ldg(src + (size_t)(compact ? m : p) * C + c));
}

// bits[pos(m)][c] = -log2(max(P, 1e-9)) of ydec under N(mean, scale)
__device__ __forceinline__ void bits_item(const int* pos, int C, const int32_t* ydec,
                                          const float* mean, const float* scale, float* bits,
                                          long idx) {
  const int m = idx / C, c = idx % C;
  const size_t o = (size_t)map_row(pos, m) * C + c;
  stg(bits + o, symbol_bits_of(ldg(ydec + o), ldg(mean + o), ldg(scale + o)));
}

}  // namespace dev
}  // namespace pswa
