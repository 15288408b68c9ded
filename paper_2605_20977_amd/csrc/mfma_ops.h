// Low-precision GEMM tile on gfx950 matrix cores (MFMA), shared by the
// per-launch kernels and the persistent decode kernel.
//
// Projections and MLP run as BF16 or FP8 (OCP e4m3fn) products with FP32
// accumulation; everything else (norm statistics, softmax, accumulator
// attention, head nonlinearity, CDF selection) stays FP32.
//
// Tile: 32 A rows (two 16-row MFMA blocks) x 64 weight rows (16 per wave).
//   1. row statistics, one wave per row, lane l over the row's float4 chunks
//      l, l+64, ... in order: sum of squares (RMSNorm) through a fixed xor
//      tree, and the row's absolute maximum after the gain (FP8 scale);
//   2. from the same registers the wave stages the row, times the gain
//      (RMSNorm input) or the input scale (integer latents), as BF16 (round
//      to nearest even) or as FP8 (round to nearest even, saturating) of
//      either value * 448 / row max (per-row scale) or value * 1/rms *
//      ascale (static per-tensor scale of the projection input, calibrated
//      offline), in LDS with a 16-byte skew per row;
//   3. each wave runs v_mfma_f32_16x16x32_{bf16,fp8_fp8} over k = 0, 32, ...
//      in order for its 16 weight rows (16 k-steps of weight loads in flight
//      at a time; the first of them issued right after the first row loads,
//      so the weight fetch overlaps steps 1 and 2) against both row blocks:
//      an output is one MFMA chain over K, whatever the tiling;
//   4. the epilogue rescales (1/rms and row max / 448, or 1 / ascale; and
//      1 / weight scale) and applies the same epilogues as the FP32 tile.
// A row's result depends only on that row, K and the weights: the same in
// every launch shape, so encode and decode stay bit-identical.
// Paired epilogues: columns 0-7 of a wave are W rows n..n+7 and columns 8-15
// the W2 rows n..n+7; lane l (column < 8) takes its partner from lane l + 8.
//
// Weight layout (the library's BF16 / FP8 copies of a [N][K] weight; N a
// multiple of 8, K of 32): units of 8 rows; inside a unit, blocks of one
// k-step (32 columns) in k order; inside a block, 32 chunks of 8 consecutive
// k values, chunk (8 * kg + row % 8) holding row (row % 8), columns
// 8 kg .. 8 kg + 7 of the k-step. Element (n, k) sits at
//   ((n / 8 * K / 32 + k / 32) * 32 + 8 * (k % 32 / 8) + n % 8) * 8 + k % 8.
// A wave's load of one k-step for 16 rows (or 8 W and 8 W2 rows) is then
// two contiguous 256-element blocks instead of 16 strided row pieces, and
// rows 8u .. 8u + 7 keep the span of the row-major layout, so a weight that
// starts at a row offset (a multiple of 8) is addressed the same way.
#pragma once

#include <hip/hip_runtime.h>

#include "device_ops.h"

namespace pswa {
namespace dev {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMBq = 32;        // largest A-row count of a low-precision tile
// The persistent kernel stages all A rows of a phase at once (up to
// kMBqWide of them) when K <= kWideMaxK, and runs each column tile against
// all of them with its weights loaded once.
constexpr int kMBqWide = 96;
constexpr int kWideMaxK = 512;
constexpr float kFp8Max = 448.0f;

__host__ __device__ inline int qgemm_col_tiles(int N, int epi) {
  const int per = kWaves * (paired_epi(epi) ? 8 : 16);
  return (N + per - 1) / per;
}
constexpr int kKchunk = 16;  // k-steps whose weight loads are issued together
__host__ __device__ inline int qgemm_row_tiles(int M, int R = kMBq) { return (M + R - 1) / R; }
// element pitch of a staged row: K plus a 16-byte skew
__host__ __device__ inline int qgemm_pitch(int K, int prec) { return K + (prec == PSWA_PREC_BF16 ? 8 : 16); }
// LDS of a tile: the staged A tile (kQRedBytes is a spare prefix kept for
// alignment of the tile).
constexpr size_t kQRedBytes = 256;
__host__ __device__ inline size_t qgemm_lds_bytes(int K, int prec, int R = kMBq) {
  return kQRedBytes + (size_t)R * qgemm_pitch(K, prec) * (prec == PSWA_PREC_BF16 ? 2 : 1);
}

// Operand types of the two MFMA forms: 8 BF16 or 8 FP8 values per lane
// (FP32 instances of the tile templates exist but never run).
template <int PREC> struct QOp {
  typedef long T;
  static constexpr int EB = 1;
};
template <> struct QOp<PSWA_PREC_BF16> {
  typedef bf16x8 T;
  static constexpr int EB = 2;
};
__device__ __forceinline__ f32x4 mfma_q(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma_q(long a, long b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
}
// 8 consecutive values at element offset e of a BF16 / FP8 array in global
// memory (load_w8) or in LDS (load_s8)
template <int PREC>
__device__ __forceinline__ typename QOp<PREC>::T load_w8(const void* base, size_t e) {
  return ldg(reinterpret_cast<const typename QOp<PREC>::T*>(static_cast<const uint8_t*>(base) +
                                                             e * QOp<PREC>::EB));
}
template <int PREC>
__device__ __forceinline__ typename QOp<PREC>::T load_s8(const uint8_t* lds, size_t e) {
  return *reinterpret_cast<const typename QOp<PREC>::T*>(lds + e * QOp<PREC>::EB);
}
// Element offset, in the unit layout above, of lane chunk kg of weight row n
// at k-step 0 (k-step s adds 256 s).
__device__ __forceinline__ size_t wfrag_offset(int n, int kg, int ksteps) {
  return ((size_t)(n >> 3) * ksteps) * 256 + (size_t)(8 * kg + (n & 7)) * 8;
}

// Steps 1 and 2 of a low-precision tile for rows m0 .. m0+rows-1 of A, one
// wave per row (rows wave, wave + 4, ...): lane l loads the row's float4
// chunks l, l+64, ... (CPR of them; RPB = 16 / CPR rows per wave in flight
// at once, indices clamped into the row so every load is unconditional),
//   * row statistics: the sum of squares (RMS) over the lane's chunks in
//     order, then a fixed xor tree, gives 1/rms; for per-row FP8 the absolute
//     maximum of x * g through a max tree gives the input scale 448 / max;
//   * the same registers, times the gain (RMSNorm input) or the input scale
//     (integer latents), are written to LDS as BF16 (round to nearest even)
//     or as FP8 (round to nearest even, saturating) of value * 448 / row max
//     (per row) or value * 1/rms * ascale (static per tensor), rows
//     [R][pitch] with a 16-byte skew per row.
// issue_w() runs once, right after the first batch of row loads is issued,
// so loads the caller issues there complete after (and are not waited for
// with) the row data.
template <int AK, bool RMS, int PREC, int R, int CPR, typename IssueW>
__device__ __forceinline__ void stage_rows(const GemmArgs& a, int m0, int rows, uint8_t* smem,
                                           float* rstd, float* rmul, IssueW& issue_w) {
  constexpr int RPB = 16 / CPR;
  constexpr int EB = PREC == PSWA_PREC_BF16 ? 2 : 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int K = a.K, K4 = a.K / 4;
  const int pitch = qgemm_pitch(K, PREC);
  const bool stat = PREC == PSWA_PREC_FP8 && a.ascale > 0.f;  // static per-tensor FP8 scale
  // per-column factor (gain or input scale) of the lane's chunks
  float4 gg[CPR];
#pragma unroll
  for (int it = 0; it < CPR; ++it) {
    const int cc = min(lane + 64 * it, K4 - 1);
    gg[it] = make_float4(1.f, 1.f, 1.f, 1.f);
    if (RMS) gg[it] = ldg4(a.gain + 4 * cc);
    if (AK == A_INT) gg[it] = ldg4(a.xscale + 4 * cc);
  }
  bool issued = false;
  for (int mb = 0; mb < rows; mb += RPB * kWaves) {
    float4 xs[RPB][CPR];
#pragma unroll
    for (int j = 0; j < RPB; ++j) {
      const int mm = min(mb + wave + kWaves * j, rows - 1);
      const size_t off = (size_t)map_row(a.xrow, m0 + mm) * a.ldx;
#pragma unroll
      for (int it = 0; it < CPR; ++it) {
        const int cc = min(lane + 64 * it, K4 - 1);
        if (AK == A_INT) {
          const int4 xi = ldg4(a.Xi + off + 4 * cc);
          xs[j][it] = make_float4(float(xi.x), float(xi.y), float(xi.z), float(xi.w));
        } else {
          xs[j][it] = ldg4(a.X + off + 4 * cc);
        }
      }
    }
    if (!issued) {
      issue_w();
      issued = true;
    }
#pragma unroll
    for (int j = 0; j < RPB; ++j) {
      const int mm = mb + wave + kWaves * j;
      float ss = 0.f, mx = 0.f;
#pragma unroll
      for (int it = 0; it < CPR; ++it) {
        // a chunk past K adds +0 to the sum and cannot raise the maximum
        const bool in = lane + 64 * it < K4;
        const float4 x = in ? xs[j][it] : make_float4(0.f, 0.f, 0.f, 0.f);
        if (RMS) ss = dot4(x, x, ss);
        if (PREC == PSWA_PREC_FP8 && !stat) {
          const float4 g = gg[it];
          mx = fmaxf(mx, fmaxf(fmaxf(fabsf(x.x * g.x), fabsf(x.y * g.y)),
                               fmaxf(fabsf(x.z * g.z), fabsf(x.w * g.w))));
        }
      }
      if (RMS) ss = wave_sum(ss);
      const float rs = RMS ? 1.0f / sqrtf(ss / float(K) + kEps) : 1.0f;
      // FP8 rows are stored as value * sc. Per row: sc = 448 / the row's
      // maximum (a zero row stays zero); the product is divided by sc and,
      // for RMSNorm inputs, multiplied by 1/rms. Static per tensor: sc =
      // ascale * 1/rms, so the stored values are the RMSNorm output times the
      // tensor's scale, and the product is divided by ascale alone.
      float sc = 1.0f;
      if (PREC == PSWA_PREC_FP8) {
        if (stat) {
          sc = RMS ? a.ascale * rs : a.ascale;
        } else {
          mx = wave_max(mx);
          sc = mx > 0.f ? kFp8Max / mx : 1.0f;
        }
      }
      if (mm >= rows) continue;  // the same for the whole wave
      if (lane == 0) {
        rstd[mm] = stat ? 1.0f : rs;
        rmul[mm] = stat ? a.ascale : sc;
      }
#pragma unroll
      for (int it = 0; it < CPR; ++it) {
        const int c = lane + 64 * it;
        if (c >= K4) continue;
        const float4 g = gg[it];
        const float4 x = make_float4(xs[j][it].x * g.x, xs[j][it].y * g.y, xs[j][it].z * g.z,
                                     xs[j][it].w * g.w);
        if (PREC == PSWA_PREC_BF16) {
          uint2 v;
          v.x = uint32_t(bf16_rne(x.x)) | (uint32_t(bf16_rne(x.y)) << 16);
          v.y = uint32_t(bf16_rne(x.z)) | (uint32_t(bf16_rne(x.w)) << 16);
          *reinterpret_cast<uint2*>(smem + (size_t)(mm * pitch + 4 * c) * EB) = v;
        } else {
          const float q0 = fminf(kFp8Max, fmaxf(-kFp8Max, x.x * sc));
          const float q1 = fminf(kFp8Max, fmaxf(-kFp8Max, x.y * sc));
          const float q2 = fminf(kFp8Max, fmaxf(-kFp8Max, x.z * sc));
          const float q3 = fminf(kFp8Max, fmaxf(-kFp8Max, x.w * sc));
          const int lo = __builtin_amdgcn_cvt_pk_fp8_f32(q0, q1, 0, false);
          const int hi = __builtin_amdgcn_cvt_pk_fp8_f32(q2, q3, lo, true);
          *reinterpret_cast<uint32_t*>(smem + (size_t)(mm * pitch + 4 * c)) = uint32_t(hi);
        }
      }
    }
  }
  if (!issued) issue_w();
}

// Steps 1 and 2 of a low-precision tile (see stage_rows); rows past the end
// of A up to R are zeros (their results are dropped). Ends with a block
// barrier.
template <int AK, bool RMS, int PREC, int R, typename IssueW>
__device__ __forceinline__ void stage_a(const GemmArgs& a, int m0, int rows, uint8_t* smem,
                                        float* rstd, float* rmul, IssueW& issue_w) {
  const int K4 = a.K / 4;
  const int cpr = (K4 + 63) / 64;  // float4 chunks per row and lane
  if (cpr <= 1) stage_rows<AK, RMS, PREC, R, 1>(a, m0, rows, smem, rstd, rmul, issue_w);
  else if (cpr <= 2) stage_rows<AK, RMS, PREC, R, 2>(a, m0, rows, smem, rstd, rmul, issue_w);
  else if (cpr <= 4) stage_rows<AK, RMS, PREC, R, 4>(a, m0, rows, smem, rstd, rmul, issue_w);
  else stage_rows<AK, RMS, PREC, R, 8>(a, m0, rows, smem, rstd, rmul, issue_w);
  // zero rows past the end of A (whole 8-byte words of each padding row)
  const int pitch_b = qgemm_pitch(a.K, PREC) * (PREC == PSWA_PREC_BF16 ? 2 : 1);
  const int words = (R - rows) * pitch_b / 8;
  for (int i = threadIdx.x; i < words; i += kThreads)
    reinterpret_cast<uint2*>(smem + (size_t)rows * pitch_b)[i] = make_uint2(0u, 0u);
  __syncthreads();
}

// R = A rows per tile (16 or 32, one or two 16-row MFMA blocks); a row
// always sits at position (row % 16) of its MFMA block, so R changes which
// tile computes a row, never how. stage = false reuses the A tile (and its
// row statistics) this block staged for the same row tile just before.
// KS = K / 32 when known at compile time (0: read from the arguments); a
// compile-time count lets the k loop run without branches, so its LDS reads
// are issued ahead of the MFMAs. CB = groups of 16 weight rows per wave (a
// wider tile: fewer tiles per block, each A fragment read once for all
// groups). The arithmetic of an output is the same for every KS and CB.
template <int AK, bool RMS, int EPI, int PREC, int R = kMBq, int KS = 0, int CB = 1>
__device__ __forceinline__ void gemm_tile_q(const GemmArgs& a, int bx, int by, uint8_t* lds, float* rstd,
                            float* rmul, bool stage = true) {
  uint8_t* smem = lds + kQRedBytes;
  constexpr bool PAIRED = paired_epi(EPI);
  constexpr int RB = R / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int K = a.K;
  const int pitch = qgemm_pitch(K, PREC);
  const int m0 = by * R;
  const int rows = min(R, a.M - m0);
  // a tile that stages waits until the block's previous tile is done with
  // the LDS; one that reuses the staged rows writes nothing shared, so its
  // waves run on without a block barrier
  if (stage) __syncthreads();

  // 3. MFMA over K for this wave's CB groups of 16 weight rows (8 W and 8
  // W2 rows per group for the paired epilogues)
  typedef typename QOp<PREC>::T WT;
  const int col = lane & 15, kg = lane >> 4;
  const int per_wave = (PAIRED ? 8 : 16) * CB;
  const int nbase = bx * kWaves * per_wave + wave * per_wave;
  const int ksteps = KS ? KS : K / 32;
  constexpr bool kFull = KS > 0 && KS % kKchunk == 0;  // every chunk complete
  size_t wofs[CB];
  const void* wbase[CB];
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    int wn;  // weight row this lane streams for group c
    if (PAIRED) {
      wn = min(nbase + 8 * c + (col & 7), a.N - 1);
      wbase[c] = col < 8 ? a.Wq : a.W2q;
    } else {
      wn = min(nbase + 16 * c + col, a.N - 1);
      wbase[c] = a.Wq;
    }
    wofs[c] = wfrag_offset(wn, kg, ksteps);
  }
  // weight loads of the first chunk and the residual inputs of this lane's
  // outputs: issued right after the A rows' first loads (or at once when
  // the staged rows are reused)
  WT b[CB][kKchunk];
  float rres[CB][RB][4];
  auto issue_w = [&]() {
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
      for (int u = 0; u < kKchunk; ++u)
        if (u < ksteps) b[c][u] = load_w8<PREC>(wbase[c], wofs[c] + 256 * u);
    if constexpr (EPI == EPI_RESID) {
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        const int nc = min(nbase + 16 * c + col, a.N - 1);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int row = m0 + min(16 * rb + 4 * kg + i, rows - 1);
            rres[c][rb][i] = ldg(a.R + (size_t)map_row(a.rrow, row) * a.ldr + nc);
          }
      }
    }
  };
  if (stage)
    stage_a<AK, RMS, PREC, R>(a, m0, rows, smem, rstd, rmul, issue_w);
  else
    issue_w();

  f32x4 acc[CB][RB];
#pragma unroll
  for (int c = 0; c < CB; ++c)
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) acc[c][rb] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < ksteps; k0 += kKchunk) {
    if (k0 > 0) {
#pragma unroll
      for (int c = 0; c < CB; ++c)
#pragma unroll
        for (int u = 0; u < kKchunk; ++u)
          if (kFull || k0 + u < ksteps) b[c][u] = load_w8<PREC>(wbase[c], wofs[c] + 256 * (k0 + u));
    }
    // A fragments of 4 k-steps read from LDS together, then their MFMAs
#pragma unroll
    for (int u0 = 0; u0 < kKchunk; u0 += 4) {
      WT af[RB][4];
#pragma unroll
      for (int u = u0; u < u0 + 4; ++u) {
        if (kFull || k0 + u < ksteps) {
          const int k = 32 * (k0 + u) + 8 * kg;
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
            af[rb][u - u0] = load_s8<PREC>(smem, (size_t)(16 * rb + col) * pitch + k);
        }
      }
#pragma unroll
      for (int u = u0; u < u0 + 4; ++u) {
        if (kFull || k0 + u < ksteps) {
#pragma unroll
          for (int c = 0; c < CB; ++c)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
              acc[c][rb] = mfma_q(af[rb][u - u0], b[c][u], acc[c][rb]);
        }
      }
    }
  }

  // 4. epilogue: lane holds rows 16*rb + 4*kg + i of its column; the row
  // scales are read from LDS and the W2 partners exchanged for all of the
  // lane's outputs first
  const float wsc = (PAIRED && col >= 8) ? a.w2scale : a.wscale;
  float rsc[RB][4], rst[RB][4];  // the rows' FP8 input scales and 1/rms
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int mrc = min(16 * rb + 4 * kg + i, rows - 1);
      rsc[rb][i] = PREC == PSWA_PREC_FP8 ? rmul[mrc] : 1.0f;
      rst[rb][i] = RMS ? rstd[mrc] : 1.0f;
    }
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    float vv[RB][4], v2v[RB][4];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float v = acc[c][rb][i] * wsc;
        if (PREC == PSWA_PREC_FP8) v = v / rsc[rb][i];
        if (RMS) v *= rst[rb][i];
        vv[rb][i] = v;
      }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        v2v[rb][i] = PAIRED ? __shfl(vv[rb][i], (lane & ~15) | ((col + 8) & 15), 64) : 0.f;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int mr = 16 * rb + 4 * kg + i;
        if (mr >= rows) continue;
        if (PAIRED && col >= 8) continue;
        const int row = m0 + mr;
        const int n = PAIRED ? nbase + 8 * c + col : nbase + 16 * c + col;
        if (n >= a.N) continue;
        if constexpr (EPI == EPI_RESID)
          stg(a.Y + (size_t)map_row(a.yrow, row) * a.ldy + n, rres[c][rb][i] + vv[rb][i]);
        else
          epilogue<EPI>(a, row, n, vv[rb][i], v2v[rb][i]);
      }
    }
  }
}

// A column tile against every row of a phase whose A rows (all M <= 96 of
// them, K <= 512) the block has staged once in LDS (stage_a with R = 96):
// each wave's weight rows for all k-steps (K / 32 <= kKchunk) are loaded
// once into b (coltile_weights), and the R-row tiles 0 .. rt - 1 run with
// them in turn. Every output's arithmetic is gemm_tile_q's: the same MFMA
// chain over the k-steps in order from zero, the same row statistics,
// scales and epilogue.
template <int EPI, int PREC, int KS>
__device__ __forceinline__ void coltile_weights(const GemmArgs& a, int bx,
                                                typename QOp<PREC>::T (&b)[kKchunk]) {
  constexpr bool PAIRED = paired_epi(EPI);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, kg = lane >> 4;
  const int per_wave = PAIRED ? 8 : 16;
  const int nbase = bx * kWaves * per_wave + wave * per_wave;
  const int ksteps = KS ? KS : a.K / 32;
  const void* wb;
  int wn;
  if (PAIRED) {
    wn = min(nbase + (col & 7), a.N - 1);
    wb = col < 8 ? a.Wq : a.W2q;
  } else {
    wn = min(nbase + col, a.N - 1);
    wb = a.Wq;
  }
  const size_t wofs = wfrag_offset(wn, kg, ksteps);
#pragma unroll
  for (int u = 0; u < kKchunk; ++u)
    if (u < ksteps) b[u] = load_w8<PREC>(wb, wofs + 256 * u);
}
template <int AK, bool RMS, int EPI, int PREC, int R, int KS>
__device__ __forceinline__ void gemm_coltile_q(const GemmArgs& a, int bx, int rt, uint8_t* lds,
                                               const float* rstd, const float* rmul,
                                               const typename QOp<PREC>::T (&b)[kKchunk]) {
  const uint8_t* smem = lds + kQRedBytes;
  constexpr bool PAIRED = paired_epi(EPI);
  constexpr int RB = R / 16;
  constexpr int kMaxRt = kMBqWide / R;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int pitch = qgemm_pitch(a.K, PREC);
  typedef typename QOp<PREC>::T WT;
  const int col = lane & 15, kg = lane >> 4;
  const int per_wave = PAIRED ? 8 : 16;
  const int nbase = bx * kWaves * per_wave + wave * per_wave;
  const int ksteps = KS ? KS : a.K / 32;
  const float wsc = (PAIRED && col >= 8) ? a.w2scale : a.wscale;
  const int n = nbase + col;
#pragma unroll
  for (int r = 0; r < kMaxRt; ++r) {
    if (r >= rt) break;  // the same for the whole block
    const int m0 = r * R;
    const int rows = min(R, a.M - m0);
    float rres[RB][4];
    if constexpr (EPI == EPI_RESID) {
      const int nc = min(n, a.N - 1);
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = m0 + min(16 * rb + 4 * kg + i, rows - 1);
          rres[rb][i] = ldg(a.R + (size_t)map_row(a.rrow, row) * a.ldr + nc);
        }
    }
    f32x4 acc[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) acc[rb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int u0 = 0; u0 < kKchunk; u0 += 4) {
      WT af[RB][4];
#pragma unroll
      for (int u = u0; u < u0 + 4; ++u) {
        if (u < ksteps) {
          const int k = 32 * u + 8 * kg;
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
            af[rb][u - u0] = load_s8<PREC>(smem, (size_t)(m0 + 16 * rb + col) * pitch + k);
        }
      }
#pragma unroll
      for (int u = u0; u < u0 + 4; ++u) {
        if (u < ksteps) {
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) acc[rb] = mfma_q(af[rb][u - u0], b[u], acc[rb]);
        }
      }
    }
    float vv[RB][4], v2v[RB][4];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int mrc = m0 + min(16 * rb + 4 * kg + i, rows - 1);
        float v = acc[rb][i] * wsc;
        if (PREC == PSWA_PREC_FP8) v = v / rmul[mrc];
        if (RMS) v *= rstd[mrc];
        vv[rb][i] = v;
      }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        v2v[rb][i] = PAIRED ? __shfl(vv[rb][i], (lane & ~15) | ((col + 8) & 15), 64) : 0.f;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int mr = 16 * rb + 4 * kg + i;
        if (mr >= rows) continue;
        if (PAIRED && col >= 8) continue;
        if (n >= a.N) continue;
        const int row = m0 + mr;
        if constexpr (EPI == EPI_RESID)
          stg(a.Y + (size_t)map_row(a.yrow, row) * a.ldy + n, rres[rb][i] + vv[rb][i]);
        else
          epilogue<EPI>(a, row, n, vv[rb][i], v2v[rb][i]);
      }
    }
  }
}

// Column tiles of a small tile with CB groups per wave.
__host__ __device__ inline int qgemm_col_tiles_cb(int N, int epi, int cb) {
  const int per = kWaves * (paired_epi(epi) ? 8 : 16) * cb;
  return (N + per - 1) / per;
}

// Large-M tile: R A rows x (kWaves * CB * 16) weight rows per block. Each
// wave computes all R rows for CB groups of 16 weight rows (8 W and 8 W2
// rows per group for the paired epilogues), every A fragment read from LDS
// once for its CB groups. Per output the arithmetic is exactly the small
// tile's: the same MFMA chain over the k-steps in order from zero, the same
// row statistics, scales and epilogue, so results never depend on which
// tile computed them.
template <int AK, bool RMS, int EPI, int PREC, int R, int CB, int KS = 0>
__device__ __forceinline__ void gemm_tile_qb(const GemmArgs& a, int bx, int by, uint8_t* lds,
                                             float* rstd, float* rmul) {
  uint8_t* smem = lds + kQRedBytes;
  constexpr bool PAIRED = paired_epi(EPI);
  constexpr int RB = R / 16;
  constexpr int KC = 4;  // k-steps whose weight loads are issued together
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int K = a.K;
  const int pitch = qgemm_pitch(K, PREC);
  const int m0 = by * R;
  const int rows = min(R, a.M - m0);
  typedef typename QOp<PREC>::T WT;
  const int col = lane & 15, kg = lane >> 4;
  const int per_wave = (PAIRED ? 8 : 16) * CB;
  const int nbase = bx * kWaves * per_wave + wave * per_wave;
  const int ksteps = KS ? KS : K / 32;
  constexpr bool kFull = KS > 0 && KS % KC == 0;  // every chunk complete
  size_t wofs[CB];
  const void* wb[CB];
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    int wn;
    if (PAIRED) {
      wn = min(nbase + 8 * c + (col & 7), a.N - 1);
      wb[c] = col < 8 ? a.Wq : a.W2q;
    } else {
      wn = min(nbase + 16 * c + col, a.N - 1);
      wb[c] = a.Wq;
    }
    wofs[c] = wfrag_offset(wn, kg, ksteps);
  }
  // the first chunk of weight loads, issued right after the A rows' first loads
  WT b[KC][CB];
  auto issue_w = [&]() {
#pragma unroll
    for (int u = 0; u < KC; ++u)
#pragma unroll
      for (int c = 0; c < CB; ++c)
        if (u < ksteps) b[u][c] = load_w8<PREC>(wb[c], wofs[c] + 256 * u);
  };
  stage_a<AK, RMS, PREC, R>(a, m0, rows, smem, rstd, rmul, issue_w);

  f32x4 acc[RB][CB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int c = 0; c < CB; ++c) acc[rb][c] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < ksteps; k0 += KC) {
    if (k0 > 0) {
#pragma unroll
      for (int u = 0; u < KC; ++u)
#pragma unroll
        for (int c = 0; c < CB; ++c)
          if (kFull || k0 + u < ksteps) b[u][c] = load_w8<PREC>(wb[c], wofs[c] + 256 * (k0 + u));
    }
#pragma unroll
    for (int u = 0; u < KC; ++u) {
      if (!kFull && k0 + u >= ksteps) continue;
      const int k = 32 * (k0 + u) + 8 * kg;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const WT af = load_s8<PREC>(smem, (size_t)(16 * rb + col) * pitch + k);
#pragma unroll
        for (int c = 0; c < CB; ++c) acc[rb][c] = mfma_q(af, b[u][c], acc[rb][c]);
      }
    }
  }

  const float wsc = (PAIRED && col >= 8) ? a.w2scale : a.wscale;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
    for (int c = 0; c < CB; ++c) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int mr = 16 * rb + 4 * kg + i;
        const int mrc = min(mr, rows - 1);
        float v = acc[rb][c][i] * wsc;
        if (PREC == PSWA_PREC_FP8) v = v / rmul[mrc];
        if (RMS) v *= rstd[mrc];
        const float v2 = PAIRED ? __shfl(v, (lane & ~15) | ((col + 8) & 15), 64) : 0.f;
        if (mr >= rows) continue;
        if (PAIRED && col >= 8) continue;
        const int n = PAIRED ? nbase + 8 * c + col : nbase + 16 * c + col;
        if (n >= a.N) continue;
        epilogue<EPI>(a, m0 + mr, n, v, v2);
      }
    }
  }
}

__host__ __device__ inline int qgemm_big_col_tiles(int N, int epi, int cb) {
  const int per = kWaves * (paired_epi(epi) ? 8 : 16) * cb;
  return (N + per - 1) / per;
}

// Runtime K to the compile-time k-step counts of the model shapes in use
// (K = 128, 192, 384, 512, 1536); other K run the generic loop.
#define PSWA_KS_DISPATCH_WIDE(K, CALL) \
  switch ((K) / 32) {                  \
    case 4: CALL(4); break;            \
    case 6: CALL(6); break;            \
    case 12: CALL(12); break;          \
    case 16: CALL(16); break;          \
    default: CALL(0); break;           \
  }
#define PSWA_KS_DISPATCH(K, CALL) \
  switch ((K) / 32) {             \
    case 4: CALL(4); break;       \
    case 6: CALL(6); break;       \
    case 12: CALL(12); break;     \
    case 16: CALL(16); break;     \
    case 48: CALL(48); break;     \
    default: CALL(0); break;      \
  }

template <int AK, bool RMS, int EPI, int R = kMBq>
__device__ __forceinline__ void gemm_tile_q_any(const GemmArgs& a, int bx, int by, uint8_t* lds,
                                                float* rstd, float* rmul, bool stage = true) {
#define PSWA_TILE_BF16(KSV) \
  gemm_tile_q<AK, RMS, EPI, PSWA_PREC_BF16, R, KSV>(a, bx, by, lds, rstd, rmul, stage)
#define PSWA_TILE_FP8(KSV) \
  gemm_tile_q<AK, RMS, EPI, PSWA_PREC_FP8, R, KSV>(a, bx, by, lds, rstd, rmul, stage)
  if (a.prec == PSWA_PREC_BF16) {
    PSWA_KS_DISPATCH(a.K, PSWA_TILE_BF16)
  } else {
    PSWA_KS_DISPATCH(a.K, PSWA_TILE_FP8)
  }
#undef PSWA_TILE_BF16
#undef PSWA_TILE_FP8
}

}  // namespace dev
}  // namespace pswa
