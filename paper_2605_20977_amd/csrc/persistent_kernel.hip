// Persistent wavefront decode kernel: one launch walks every diagonal of a
// batch of frames (of any sizes, I and P mixed). The frames are split into
// groups, each served by its own blocks; at step t a group's rows are the
// union of its frames' diagonal t, each phase of the network (see network.h)
// is spread over the group's blocks as GEMM tiles or attention items, and the
// group's blocks meet at the group's barrier between dependent phases.
//
// The barrier is a monotonic arrival counter in device memory: a block's
// leader adds one arrival with release semantics (publishing the block's
// writes) and spins with acquire loads, a bounded number of times, until
// every block of the group has arrived. Its cost grows with the number of
// blocks that share it (about 1 us at 16 blocks and 10 us at 256 on MI355X),
// which is why groups are kept small. If the bound is ever exceeded (a block
// that is not co-resident, say), the leader raises the abort flag; every
// block leaves at its next barrier, so the kernel always drains and the host
// reports the abort.
//
// This file is compiled once per instance: PSWA_PREC, PSWA_DH and PSWA_R
// name the projection arithmetic, head size and row-tile height, and the
// instance is reached through pswa_persistent_kernel_<PREC>_<DH>_<R>().
#include <hip/hip_runtime.h>

#include "device_ops.h"
#include "mfma_ops.h"
#include "network.h"
#include "persistent.h"

#if !defined(PSWA_PREC) || !defined(PSWA_DH) || !defined(PSWA_R)
#error "compile with -DPSWA_PREC=<0|1|2> -DPSWA_DH=<16|32|48|64> -DPSWA_R=<16|32>"
#endif

namespace pswa {

using namespace dev;

namespace {

// Barrier of the nb blocks of one group. Two forms of the same arrival
// counter (bounded spin, abort flag):
//  * device scope (any placement): the arrival is a release and the poll an
//    acquire at agent scope, which write the XCD's L2 back and invalidate it;
//  * one XCD (every block of the group verified to run on the same XCD):
//    each wave waits until its stores have reached the shared L2 (no L2
//    write-back), the arrival and the poll are relaxed, and after the wait
//    the vector caches are invalidated at device scope.
__device__ __forceinline__ bool group_barrier(unsigned* bar, unsigned& target, int nb,
                                              int* abort_flag, long spin_limit, bool one_xcd) {
  __shared__ int s_ok;
  if (one_xcd) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    target += nb;
    if (one_xcd) {
      __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      // release: this block's writes become visible before its arrival counts
      __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    int ok = 1;
    long spins = 0;
    for (;;) {
      // acquire (device form): once every arrival is seen, every block's
      // writes are visible
      const unsigned seen = one_xcd
          ? __hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
          : __hip_atomic_load(bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
      if (seen >= target) break;
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
  if (one_xcd) asm volatile("buffer_inv sc1" ::: "memory");
  return s_ok != 0;
}

// Hardware id of the XCD running this wave.
__device__ __forceinline__ int xcd_id() {
  unsigned v;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
  return int(v & 0xf);
}

template <int AK, bool RMS, int EPI, int PREC, int R>
__device__ __forceinline__ void gemm_phase(const GemmArgs& a, float4* smem4, float* rstd,
                                           int rank, int nb) {
  __shared__ float rmul[kMBqWide];
  if constexpr (PREC != PSWA_PREC_F32) {
    const int rt = qgemm_row_tiles(a.M, R);
    // 16-row instances: when a phase has several row tiles (K <= 512, at
    // most 96 rows) and the column tiles spread over the blocks as evenly as
    // the tiles would, every row is staged once and each of the block's
    // column tiles runs against all of them with its weights loaded once
    // (measured faster there; slower in the 32-row instances, which keep the
    // row-tile-major path below)
    if constexpr (R == 16) {
      const int ct = qgemm_col_tiles(a.N, EPI);
      if (rt > 1 && a.M <= kMBqWide && a.K <= kWideMaxK &&
          (ct + nb - 1) / nb * rt <= (ct * rt + nb - 1) / nb) {
        uint8_t* lds = reinterpret_cast<uint8_t*>(smem4);
        typedef typename QOp<PREC>::T WT;
        auto none = [] {};
        stage_a<AK, RMS, PREC, kMBqWide>(a, 0, a.M, lds + kQRedBytes, rstd, rmul, none);
#define PSWA_COLS(KSV)                                                          \
  for (int c = rank; c < ct; c += nb) {                                         \
    WT w[kKchunk];                                                              \
    coltile_weights<EPI, PREC, KSV>(a, c, w);                                   \
    gemm_coltile_q<AK, RMS, EPI, PREC, R, KSV>(a, c, rt, lds, rstd, rmul, w);   \
  }
        PSWA_KS_DISPATCH_WIDE(a.K, PSWA_COLS)
#undef PSWA_COLS
        return;
      }
    }
    // tiles in row-tile-major order: a block re-stages A only when its next
    // tile starts a new row tile
#define PSWA_TILES(KSV)                                                                        \
  {                                                                                            \
    const int ct = qgemm_col_tiles(a.N, EPI);                                                  \
    int staged = -1;                                                                           \
    for (int t = rank; t < ct * rt; t += nb) {                                                 \
      const int r = t / ct;                                                                    \
      gemm_tile_q<AK, RMS, EPI, PREC, R, KSV>(a, t % ct, r, reinterpret_cast<uint8_t*>(smem4), \
                                              rstd, rmul, r != staged);                        \
      staged = r;                                                                              \
    }                                                                                          \
  }
    PSWA_KS_DISPATCH(a.K, PSWA_TILES)
#undef PSWA_TILES
  } else {
    const int ct = gemm_col_tiles(a.N, EPI), rt = gemm_row_tiles(a.M);
    for (int t = rank; t < ct * rt; t += nb)
      gemm_tile_any<AK, RMS, EPI>(a, t % ct, t / ct, smem4, rstd);
  }
}

// Items (row, head pair) in head-major order (item = pair * M + row): a wave
// takes a contiguous run of them, so its consecutive items are adjacent rows
// of one head pair, whose key windows overlap (their K/V rows are then still
// in cache). The positions and frames of up to 8 items are read together
// before they run, with scalar loads from the launch's read-only row and
// frame tables (all positions, then all frames: two round trips per 8
// items), so an item waits only on its own keys. KV16: BF16 caches.
template <int DH, bool KV16>
__device__ __forceinline__ void attn_phase(const AttnArgs& a, int rank, int nb) {
  constexpr int PF = 8;
  const int items = a.M * attn_pairs(a.heads);
  const int nw = nb * kWaves;
  const int per = (items + nw - 1) / nw;
  const int i0 = __builtin_amdgcn_readfirstlane(
      min(items, (rank * kWaves + (int)(threadIdx.x >> 6)) * per));
  const int i1 = min(items, i0 + per);
  for (int b0 = i0; b0 < i1; b0 += PF) {
    int gp[PF], fr[PF], qr[PF];
    FrameInfo fi[PF];
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int m = min(b0 + i, i1 - 1) % a.M;
      gp[i] = a.pos ? load_uniform(a.pos + m) : m;
      fr[i] = a.fid ? load_uniform(a.fid + m) : 0;
      qr[i] = a.qrow ? load_uniform(a.qrow + m) : m;
    }
#pragma unroll
    for (int i = 0; i < PF; ++i) fi[i] = a.fid ? load_uniform(a.frames + fr[i]) : a.frame0;
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int item = b0 + i;
      if (item >= i1) break;  // uniform across the wave
      attn_pair_at<DH, KV16>(a, item % a.M, item / a.M, gp[i], fi[i], qr[i]);
    }
  }
}

// Rows of a per-group RMSNorm (a Channel Transformer row description: a.M
// rows, slice of a.K values at column a.nsplit of X, gain and Y) spread over
// the group's waves; the row arithmetic is the per-launch kernel's.
__device__ __forceinline__ void rms_phase(const GemmArgs& a, int rank, int nb) {
  const int nw = nb * kWaves;
  for (int m = rank * kWaves + (int)(threadIdx.x >> 6); m < a.M; m += nw)
    group_rms_row(a.X + (size_t)m * a.ldx + a.nsplit, a.gain + a.nsplit,
                  a.Y + (size_t)m * a.ldy + a.nsplit, a.K);
}

// Direct global-to-LDS loads (gfx950): every active lane moves `bytes` from
// its own global address to lds + lane * bytes (lds: the same in the wave).
__device__ __forceinline__ void lds_load16(const float* src, float* lds) {
  __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                   (__attribute__((address_space(3))) void*)lds, 16, 0, 0);
}
__device__ __forceinline__ void lds_load4(const float* src, float* lds) {
  __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                   (__attribute__((address_space(3))) void*)lds, 4, 0, 0);
}

// Keys of a staged tile: window cells and the null slot from LDS (cell slot
// of kStageCellBytes, data 16 (cell mod 8) bytes in, head hh's K then V row,
// FP32 or BF16 as the caches hold them), temporal keys of P-frames from
// global memory.
template <int DH, bool KV16>
struct StagedKeys {
  struct Slot {
    int cell;  // -1: a temporal key, in raw
    KeyRaw<DH> raw;
  };
  const AttnArgs& a;
  const float* smem;
  const float* btile;
  const int *s_base, *s_c0;
  int hd, hh, wave, pi, pj, n_sp, cells;
  FrameInfo fi;
  __device__ __forceinline__ bool issue(int kk, bool want, Slot& sl) {
    sl.cell = 0;  // unused slots read cell 0, which is never used
    sl.raw.b = 0.f;
    if (!want) return false;
    if (kk < n_sp) {
      int da, db;
      window_offset(a, kk, da, db);
      const int ki = pi + da, kj = pj + db;
      if (ki < 0 || ki >= fi.H || kj < 0 || kj >= fi.W) return false;
      const int k = wave + a.r + da;  // the key's image row within the tile
      sl.cell = s_base[k] + kj - s_c0[k];
      sl.raw.b = btile[hh * 64 + kk];
      return true;
    }
    if (a.knull && kk == n_sp) {
      sl.cell = cells;
      sl.raw.b = 0.f;
      return true;
    }
    SlotAddr s;
    if (!slot_addr(a, kk, hd, DH, pi, pj, fi, n_sp, 0, s)) return false;
    sl.cell = -1;
    sl.raw.b = ldg(a.bias + s.bias);
    kv_issue<DH, KV16>(a.tkv, s.e, a.d, sl.raw);  // temporal keys only
    return true;
  }
  __device__ __forceinline__ void get(const Slot& sl, float4* kr, float4* vr, float& b) {
    b = sl.raw.b;
    if (sl.cell < 0) {
      kv_widen<DH, KV16>(sl.raw, kr, vr);
      return;
    }
    const float* p = smem + sl.cell * (kStageCellBytes / 4) + 4 * (sl.cell & 7);
    if constexpr (KV16) {
      const int4* q = reinterpret_cast<const int4*>(reinterpret_cast<const uint16_t*>(p) +
                                                    hh * 2 * DH);
      KeyRaw<DH> r;
#pragma unroll
      for (int c = 0; c < DH / 8; ++c) {
        r.k[c] = q[c];
        r.v[c] = q[DH / 8 + c];
      }
      kv_widen<DH, true>(r, kr, vr);
    } else {
      p += hh * 2 * DH;
#pragma unroll
      for (int e = 0; e < DH / 4; ++e) {
        kr[e] = *reinterpret_cast<const float4*>(p + 4 * e);
        vr[e] = *reinterpret_cast<const float4*>(p + DH + 4 * e);
      }
    }
  }
};

// Wavefront attention from LDS-staged window tiles (see device_ops.h): the
// phase's rows are split into contiguous runs over the group's blocks; a
// block cuts its run into tiles of up to kStageRows consecutive diagonal
// rows of one frame and, per tile and group of stage_heads heads, loads the
// union of the rows' windows (one wave load per cell), the rows' queries
// and the heads' window biases into LDS, then each wave computes its row's
// items from LDS (temporal keys of P-frames are read from global memory).
// The arithmetic of every item is attn_core's, as in every other path.
// KV16: the caches hold BF16 (element offsets as for FP32).
template <int DH, bool KV16>
__device__ __forceinline__ void attn_phase_staged(const AttnArgs& a, float* smem, int rank,
                                                  int nb) {
  constexpr int HT = stage_heads(DH, KV16);
  constexpr int EP = KV16 ? 8 : 4;           // cache elements per 16-byte piece
  constexpr int QH = 2 * DH / EP;            // 16-byte pieces of one head's K and V rows
  constexpr int CF = kStageCellBytes / 4;    // floats per cell slot
  __shared__ int s_base[kStageImgRows + 1], s_c0[kStageImgRows], s_gpos[kStageCells];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = a.r, s = r + 1, d = a.d;
  const int n_sp = attn_n_sp(a);
  float* qtile = smem + kStageQOff / 4;
  float* btile = smem + stage_bias_off(DH, KV16) / 4;
  // this lane's piece of a cell: head lh of the group, 16 bytes lq of that
  // head's K (lq < QH/2) or V row, as an element offset in the position's row
  const int lh = lane / QH, lq = lane % QH;
  const int lpart = lh * DH + (lq < QH / 2 ? EP * lq : d - DH + EP * lq);
  const int rpb = (a.M + nb - 1) / nb;
  const int m_lo = min(a.M, rank * rpb), m_hi = min(a.M, m_lo + rpb);
  for (int m0 = m_lo; m0 < m_hi;) {
    // the tile's rows: consecutive diagonal rows (i + 1, j - s) of one frame
    const int gp0 = map_row(a.pos, m0);
    const int f0 = a.fid ? ldg(a.fid + m0) : 0;
    const FrameInfo fi = attn_frame(a, m0);
    int R = 1;
    while (R < kStageRows && m0 + R < m_hi) {
      const int f = a.fid ? ldg(a.fid + m0 + R) : 0;
      if (f != f0 || map_row(a.pos, m0 + R) != gp0 + R * (fi.W - s)) break;
      ++R;
    }
    const int i0 = (gp0 - fi.off) / fi.W, j0 = (gp0 - fi.off) % fi.W;
    // union of the windows, image row by image row
    int base[kStageImgRows + 1], c0[kStageImgRows];
    {
      int acc = 0;
#pragma unroll
      for (int k = 0; k < kStageImgRows; ++k) {
        const int ii = i0 - r + k;
        int ca = 0, w = 0;
        if (k < R + r && ii >= 0) {
          const int lo = max(i0, ii), hi = min(i0 + R - 1, ii + r);
          ca = max(0, j0 - s * (hi - i0) - r);
          const int cb = min(fi.W - 1, j0 - s * (lo - i0) + r);
          w = cb >= ca ? cb - ca + 1 : 0;
        }
        base[k] = acc;
        c0[k] = ca;
        acc += w;
      }
      base[kStageImgRows] = acc;
    }
    const int cells = base[kStageImgRows];
    const int ncell = cells + (a.knull ? 1 : 0);  // the null key is cell `cells`
    // the geometry in LDS: image rows (for the items' key lookup) and the
    // global position of every cell (for the loads)
#pragma unroll
    for (int k = 0; k <= kStageImgRows; ++k)
      if ((int)threadIdx.x == k) {
        s_base[k] = base[k];
        if (k < kStageImgRows) s_c0[k] = c0[k];
      }
    if ((int)threadIdx.x < cells) {
      const int cell = threadIdx.x;
      int k = 0;
#pragma unroll
      for (int kk = 1; kk < kStageImgRows; ++kk) k += cell >= base[kk] ? 1 : 0;
      int bk = base[0], ck = c0[0];
#pragma unroll
      for (int kk = 1; kk < kStageImgRows; ++kk)
        if (k == kk) {
          bk = base[kk];
          ck = c0[kk];
        }
      s_gpos[cell] = fi.off + (i0 - r + k) * fi.W + ck + cell - bk;
    }
    __syncthreads();
    const bool live = wave < R;
    const int m = m0 + min(wave, R - 1);
    const int qr = map_row(a.qrow, m);
    const int pi = i0 + wave, pj = j0 - s * wave;
    const int n_keys = attn_n_keys(a, fi);
    for (int h0 = 0; h0 < a.heads; h0 += HT) {
      const int nh = min(HT, a.heads - h0);
      // K/V rows of the heads: cell c by wave c mod 4, 16 bytes per lane
      // (the null key and value: the cache's row after its last position)
      if (lane < nh * QH) {
        for (int c = wave; c < ncell; c += kWaves) {
          const size_t e = (size_t)(c < cells ? s_gpos[c] : a.HWt) * 2 * d + h0 * DH + lpart;
          const float* src = KV16 ? reinterpret_cast<const float*>(
                                        reinterpret_cast<const uint16_t*>(a.kv) + e)
                                  : a.kv + e;
          lds_load16(src, smem + c * CF + 4 * (c & 7));
        }
      }
      // each row's query for the heads, loaded by its own wave
      if (live && lane < nh * DH / 4)
        lds_load16(a.q + (size_t)qr * a.ldq + h0 * DH + 4 * lane, qtile + wave * HT * DH);
      // the heads' window biases, 64 floats apart
      for (int hh = wave; hh < nh; hh += kWaves)
        if (lane < n_sp) lds_load4(a.bias + (h0 + hh) * a.nbias + lane, btile + hh * 64);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
      if (live) {
        // the stage's heads in pairs, one per half-wave (keys per round as in
        // attn_pair_at: one for FP32 caches, two for BF16)
        for (int hp = 0; hp < nh; hp += 2) {
          const int hs = hp + ((threadIdx.x >> 5) & 1);
          const bool hlive = hs < nh;
          const int hh = min(hs, nh - 1);
          float4 q4[DH / 4];
#pragma unroll
          for (int e = 0; e < DH / 4; ++e)
            q4[e] = *reinterpret_cast<const float4*>(qtile + wave * HT * DH + hh * DH + 4 * e);
          StagedKeys<DH, KV16> src{a,  smem, btile, s_base, s_c0, h0 + hh, hh,
                                   wave, pi, pj, n_sp, cells, fi};
          attn_core<DH, KV16 ? 2 : 1>(q4, n_keys, hlive, src,
                                      a.out + (size_t)m * a.ldo + (h0 + hh) * DH);
        }
      }
      __syncthreads();
    }
    m0 += R;
  }
}

// PREC: the projections' arithmetic (FP32 SIMT, or BF16 / FP8 on MFMA); one
// instance per (arithmetic, head size, row tile) keeps each one's registers
// to itself.
template <int PREC, int DH, int R>
__global__ void __launch_bounds__(kThreads) k_persistent(PersistArgs P) {
  extern __shared__ float4 smem4[];
  __shared__ float rstd[kMBqWide];
  float* smem = reinterpret_cast<float*>(smem4);
  const int bm = __builtin_amdgcn_readfirstlane(ldg(P.block_map + blockIdx.x));
  const GroupInfo G = load_uniform(P.groups + (bm >> 16));
  const int rank = bm & 0xffff, nb = G.nblocks;
  const bool tracer = P.trace && bm == 0 && threadIdx.x == 0;
  const int L = P.L, na = 1 + L;
  // Channel Transformer entries (FP32 instances only)
  const int ctp = PREC == PSWA_PREC_F32 && P.ct_groups ? 1 + P.ct_groups * (3 + 4 * P.ct_blocks) : 0;
  const int ng = gemm_phases(L, ctp);
  // wavefront schedule: attention from LDS-staged window tiles, if chosen
  const bool staged = P.cycle == 0 && P.attn_staged;
  const int t_end = min(P.t_end, G.T);
  unsigned target = 0;
  int nsync = 0;
  // Placement check: every block records its XCD; after a device-scope
  // barrier the group uses the one-XCD barrier if all its blocks agree.
  bool one_xcd = false;
  {
    __shared__ int s_same;
    const int slot = (bm >> 16) * nb + rank;
    if (threadIdx.x == 0) P.xcd_tab[slot] = xcd_id();
    if (!group_barrier(G.bar, target, nb, P.abort_flag, P.spin_limit, false)) return;
    if (threadIdx.x == 0) s_same = 1;
    __syncthreads();
    const int base = (bm >> 16) * nb;
    for (int k = threadIdx.x; k < nb; k += blockDim.x)
      if (__hip_atomic_load(P.xcd_tab + base + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) !=
          __hip_atomic_load(P.xcd_tab + base, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        s_same = 0;
    __syncthreads();
    one_xcd = P.xcd_local && s_same;
  }
#define PSWA_SYNC                                                                    \
  if (tracer && 2 * nsync + 1 < P.trace_len) P.trace[2 * nsync] = wall_clock64();   \
  if (!group_barrier(G.bar, target, nb, P.abort_flag, P.spin_limit, one_xcd)) return; \
  if (tracer && 2 * nsync + 1 < P.trace_len) P.trace[2 * nsync + 1] = wall_clock64(); \
  ++nsync;

  // the step's argument copy in LDS, after the phases' work area
  uint8_t* abase = reinterpret_cast<uint8_t*>(smem4) + P.args_lds_off;
  GemmArgs* g = reinterpret_cast<GemmArgs*>(abase);
  AttnArgs* at = reinterpret_cast<AttnArgs*>(abase + step_args_gemm_bytes(L, ctp));
  SymArgs* ss = reinterpret_cast<SymArgs*>(abase + step_args_gemm_bytes(L, ctp) +
                                           step_args_attn_bytes(L));

  for (int t = P.t_begin; t < t_end; ++t) {
    // copy the step's argument entries into LDS (every wave is done with the
    // previous step's copy once it passes the barrier below)
    __syncthreads();
    copy_words_to_lds(reinterpret_cast<int*>(g),
                      reinterpret_cast<const int*>(G.gtab + (size_t)t * ng),
                      ng * (int)(sizeof(GemmArgs) / 4));
    copy_words_to_lds(reinterpret_cast<int*>(at),
                      reinterpret_cast<const int*>(G.atab + (size_t)t * na),
                      na * (int)(sizeof(AttnArgs) / 4));
    copy_words_to_lds(reinterpret_cast<int*>(ss), reinterpret_cast<const int*>(G.stab + t),
                      (int)(sizeof(SymArgs) / 4));
    __syncthreads();
    const SymArgs sy = lds_uniform(ss);
    if (sy.M == 0) continue;  // same for every block of the group

    // (g0, the accumulator's query projection, depends on the hyperprior
    // tokens only: it runs for every position before the launch)
    if (staged)
      attn_phase_staged<DH, PREC != PSWA_PREC_F32>(lds_uniform(at + 0), smem, rank, nb);
    else
      attn_phase<DH, PREC != PSWA_PREC_F32>(lds_uniform(at + 0), rank, nb);
    PSWA_SYNC
    gemm_phase<A_FLOAT, false, EPI_RESID, PREC, R>(lds_uniform(g + 1), smem4, rstd, rank, nb);
    PSWA_SYNC
    for (int l = 0; l < L; ++l) {
      gemm_phase<A_FLOAT, true, EPI_QKV, PREC, R>(lds_uniform(g + 2 + 4 * l), smem4, rstd, rank, nb);
      PSWA_SYNC
      if (staged)
        attn_phase_staged<DH, PREC != PSWA_PREC_F32>(lds_uniform(at + 1 + l), smem, rank, nb);
      else
        attn_phase<DH, PREC != PSWA_PREC_F32>(lds_uniform(at + 1 + l), rank, nb);
      PSWA_SYNC
      gemm_phase<A_FLOAT, false, EPI_RESID, PREC, R>(lds_uniform(g + 3 + 4 * l), smem4, rstd, rank, nb);
      PSWA_SYNC
      gemm_phase<A_FLOAT, true, EPI_SWIGLU, PREC, R>(lds_uniform(g + 4 + 4 * l), smem4, rstd, rank, nb);
      PSWA_SYNC
      gemm_phase<A_FLOAT, false, EPI_RESID, PREC, R>(lds_uniform(g + 5 + 4 * l), smem4, rstd, rank, nb);
      PSWA_SYNC
    }
    bool plain_head = true;
    if constexpr (PREC == PSWA_PREC_F32) {
      if (P.ct_groups) {
        // Channel Transformer: every group's input map, then group by group
        // the latent map (groups > 0), the blocks and the group's head, whose
        // epilogue gathers the group's symbols for the next group
        plain_head = false;
        const GemmArgs* ct = g + gemm_phases(L);
        gemm_phase<A_FLOAT, true, EPI_STORE, PREC, R>(lds_uniform(ct), smem4, rstd, rank, nb);
        PSWA_SYNC
        int e = 1;
        for (int gi = 0; gi < P.ct_groups; ++gi) {
          if (gi > 0) {
            gemm_phase<A_INT, false, EPI_RESID, PREC, R>(lds_uniform(ct + e), smem4, rstd, rank, nb);
            PSWA_SYNC
          }
          ++e;
          for (int bl = 0; bl < P.ct_blocks; ++bl) {
            rms_phase(lds_uniform(ct + e), rank, nb);
            PSWA_SYNC
            gemm_phase<A_FLOAT, false, EPI_RESID, PREC, R>(lds_uniform(ct + e + 1), smem4, rstd, rank, nb);
            PSWA_SYNC
            gemm_phase<A_FLOAT, true, EPI_SWIGLU, PREC, R>(lds_uniform(ct + e + 2), smem4, rstd, rank, nb);
            PSWA_SYNC
            gemm_phase<A_FLOAT, false, EPI_RESID, PREC, R>(lds_uniform(ct + e + 3), smem4, rstd, rank, nb);
            PSWA_SYNC
            e += 4;
          }
          gemm_phase<A_FLOAT, true, EPI_SILU, PREC, R>(lds_uniform(ct + e), smem4, rstd, rank, nb);
          PSWA_SYNC
          gemm_phase<A_FLOAT, false, EPI_HEAD, PREC, R>(lds_uniform(ct + e + 1), smem4, rstd, rank, nb);
          PSWA_SYNC
          e += 2;
        }
      }
    }
    if (plain_head) {
      gemm_phase<A_FLOAT, true, EPI_SILU, PREC, R>(lds_uniform(g + 2 + 4 * L), smem4, rstd, rank, nb);
      PSWA_SYNC
      // head W2: mean, scale, CDF selection, and the step's symbols and bits
      gemm_phase<A_FLOAT, false, EPI_HEAD, PREC, R>(lds_uniform(g + 3 + 4 * L), smem4, rstd, rank, nb);
      PSWA_SYNC
    }
    gemm_phase<A_INT, false, EPI_STORE, PREC, R>(lds_uniform(g + 4 + 4 * L), smem4, rstd, rank, nb);
    PSWA_SYNC
    gemm_phase<A_FLOAT, true, EPI_STORE, PREC, R>(lds_uniform(g + 5 + 4 * L), smem4, rstd, rank, nb);
    PSWA_SYNC
  }
#undef PSWA_SYNC
}

}  // namespace

#ifdef PSWA_STUB_INSTANCE
// development builds of a subset of the instances: this one is absent (the
// host reports its models as unsupported)
PSWA_PERSISTENT_GETTER(PSWA_PREC, PSWA_DH, PSWA_R) { return nullptr; }
#else
PSWA_PERSISTENT_GETTER(PSWA_PREC, PSWA_DH, PSWA_R) {
  return reinterpret_cast<const void*>(&k_persistent<PSWA_PREC, PSWA_DH, PSWA_R>);
}
#endif

}  // namespace pswa
