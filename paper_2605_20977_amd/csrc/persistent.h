// Host interface of the persistent multi-frame decode kernel.
#pragma once

#include "network.h"

namespace pswa {

// Symbols of one global step: its rows, the symbol source and the outputs.
// The kernel reads M to skip an empty step; the symbols themselves are
// gathered, and their bits computed, in the head projection's epilogue.
struct SymArgs {
  int M, C;
  const int* gpos;
  const int32_t* ysrc;
  int src_compact;
  int32_t* ydec;
  const float *mean, *scale;
  float* bits;
};

// Frames of a batch are split into groups, each served by its own set of
// blocks: a group walks the global steps of its frames (the union of their
// diagonals) and its blocks meet at the group's own barrier between
// dependent phases. Frames never read each other's data, so groups never
// wait for one another.
//
// Per step t a group runs, in order (g = GEMM table entry, a = attention
// table entry; every phase ends with the group barrier):
//   a0 acc attention (its queries, g0, are computed for every position
//   before the launch), g1 acc O,
//   per layer l: g(2+4l) QKV, a(1+l) attention, g(3+4l) O, g(4+4l) gate/up,
//                g(5+4l) down,
//   g(2+4L) head W1, g(3+4L) head W2 (whose epilogue also gathers the step's
//   symbols and their bits), g(4+4L) embed, g(5+4L) acc K/V.
// The argument tables are built on the host for every group, step and phase.
// At the start of a step every block copies the step's entries into LDS with
// one round of loads; each phase then reads its entry from LDS into scalar
// registers, so no phase waits on device memory for its arguments.
struct GroupInfo {
  const GemmArgs* gtab;    // [T][6 + 4L (+ ct_phases)]
  const AttnArgs* atab;    // [T][1 + L]
  const SymArgs* stab;     // [T]
  int T;                   // steps of the group's frames
  int nblocks;             // blocks serving the group
  unsigned* bar;           // the group's barrier arrivals (zeroed before each launch)
};

struct PersistArgs {
  const GroupInfo* groups;
  const int* block_map;    // [grid]: (group << 16) | rank of the block in its group
  int L;
  int t_begin, t_end;      // global steps run by this launch (0, T for a decode)
  int* abort_flag;         // set when a barrier wait exceeds spin_limit
  long spin_limit;
  long long* trace;        // optional: wall clock after each barrier (group 0, rank 0)
  int trace_len;
  int* xcd_tab;            // [grid]: XCD of each block, by (group, rank)
  int xcd_local;           // allow the one-XCD barrier for groups that qualify
  int args_lds_off;        // byte offset of the step's argument copy in dynamic LDS
  int cycle;               // the model's schedule (0: wavefront)
  int ct_groups, ct_blocks;  // Channel Transformer (FP32 instances; 0: the plain head)
  int attn_staged;         // wavefront attention from LDS-staged window tiles (else
                           // every key read by its lane from global memory)
};

// Kernel instances: (projection arithmetic, head size, row tile). Each is
// built as its own object from persistent_kernel.hip and reached through
// pswa_persistent_kernel_<PREC>_<DH>_<R>().
#define PSWA_PERSISTENT_INSTANCES(X)                                              \
  X(0, 16, 32) X(0, 32, 32) X(0, 48, 32) X(0, 64, 32)                             \
  X(1, 16, 16) X(1, 32, 16) X(1, 48, 16) X(1, 64, 16)                             \
  X(1, 16, 32) X(1, 32, 32) X(1, 48, 32) X(1, 64, 32)                             \
  X(2, 16, 16) X(2, 32, 16) X(2, 48, 16) X(2, 64, 16)                             \
  X(2, 16, 32) X(2, 32, 32) X(2, 48, 32) X(2, 64, 32)
#define PSWA_PERSISTENT_NAME(P_, D_, R_) pswa_persistent_kernel_##P_##_##D_##_##R_
#define PSWA_PERSISTENT_NAME_X(P_, D_, R_) PSWA_PERSISTENT_NAME(P_, D_, R_)
#define PSWA_PERSISTENT_GETTER(P_, D_, R_) const void* PSWA_PERSISTENT_NAME_X(P_, D_, R_)()

// GEMM table entries of a step: the spatial network's 6 + 4L, then for
// models with channel groups `ct` more (ct_phases).
__host__ __device__ inline int gemm_phases(int L, int ct = 0) { return 6 + 4 * L + ct; }
__host__ __device__ inline int attn_phases(int L) { return 1 + L; }
// Channel Transformer entries of a step (FP32 models): the input map of
// every group at once, then per group the latent map, per block the
// per-group RMSNorm (as a row description), mixing, gate/up and down, and
// the group's head W1 and W2.
__host__ __device__ inline int ct_phases(const NetDims& x) {
  return x.cg ? 1 + x.cg * (3 + 4 * x.cL) : 0;
}

// Dynamic LDS of the kernel: the phases' work area, then the step's
// argument copy at persistent_args_lds_offset().
size_t persistent_lds_bytes(const NetDims& x, int prec, int rtile);
size_t persistent_args_lds_offset(const NetDims& x, int prec, int rtile);
// Bytes of one step's argument copy, and its parts' offsets within it.
__host__ __device__ inline size_t align16(size_t b) { return (b + 15) & ~size_t(15); }
__host__ __device__ inline size_t step_args_gemm_bytes(int L, int ct = 0) {
  return align16(gemm_phases(L, ct) * sizeof(GemmArgs));
}
__host__ __device__ inline size_t step_args_attn_bytes(int L) { return align16(attn_phases(L) * sizeof(AttnArgs)); }
__host__ __device__ inline size_t step_args_bytes(int L, int ct = 0) {
  return step_args_gemm_bytes(L, ct) + step_args_attn_bytes(L) + align16(sizeof(SymArgs));
}
// Largest grid whose blocks can all be resident at once (0 on error).
int persistent_max_grid(const NetDims& x, int prec, int rtile);
void launch_persistent(const PersistArgs& P, const NetDims& x, int prec, int rtile, int grid,
                       hipStream_t s);
void zero_ints(int* p, int n, hipStream_t s);

}  // namespace pswa
