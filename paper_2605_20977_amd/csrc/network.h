// The network as a list of phases. One pass over a set of rows (one
// diagonal of one or many frames, or every position of a frame) runs
//   accumulator: q GEMM -> window attention (+ null slot) -> O GEMM (+ h)
//   per layer:   QKV GEMM -> window attention -> O GEMM (+ residual)
//                -> gate/up SwiGLU GEMM -> down GEMM (+ residual)
//   head:        W1 GEMM (SiLU) -> W2 GEMM (mean, scale, CDF selection)
//   symbols:     gather the diagonal's symbols, their bits
//   embedding:   W_in GEMM -> accumulator K/V GEMM
// The argument builders below are __host__ __device__: the per-launch path
// calls them on the host, the persistent kernel on the device, so both run
// the same arithmetic on the same operands.
#pragma once

#include "pswa_internal.h"

namespace pswa {

constexpr int kMaxLayers = 16;

// A projection weight in the model's GEMM precision: the BF16 / FP8 copy and
// 1 / its quantization scale (FP8; 1 for BF16). q is null for FP32 models.
// ascale: the FP8 static activation scale of the projection's input (0: per
// row); slot: the input's index among the model's projection inputs (its
// calibration record).
struct QW {
  const void* q = nullptr;
  float inv_scale = 1.f;
  float ascale = 0.f;
  int slot = -1;
};

struct LayerWeights {
  const float *g1, *Wqkv, *bias, *Wo, *g2, *Wgate, *Wup, *Wdown;
  QW qkv, o, gate, up, down;
};

// Channel Transformer (models with channel groups): FP32 weights in the
// blob, plus per-group compacted copies of the masked maps made at upload:
// wy_g[g] = the shifted latent input rows of group g, [dg][g * Cg] (latent
// groups 0 .. g-1; null for g = 0), m_g[b][g] = block b's mixing rows of
// group g, [dg][(g + 1) * dg].
constexpr int kMaxChGroups = 8;
constexpr int kMaxChBlocks = 4;
struct CtWeights {
  const float *gx, *Wx, *gy, *Wy;
  const float *g1[kMaxChBlocks], *M[kMaxChBlocks], *g2[kMaxChBlocks];
  const float *Wgate[kMaxChBlocks], *Wup[kMaxChBlocks], *Wdown[kMaxChBlocks];
  const float *hg, *W1, *W2;
  const float* wy_g[kMaxChGroups];
  const float* m_g[kMaxChBlocks][kMaxChGroups];
};

struct DevWeights {
  const float *hyperW, *P4, *ing, *inW, *acc_gq, *acc_Wq, *acc_gkv, *acc_Wkv, *knull, *vnull,
      *acc_bias, *acc_Wo;
  LayerWeights layers[kMaxLayers];
  const float *head_g, *W1, *W2, *gmu, *bmu, *gsig, *bsig;
  int prec;  // PSWA_PREC_*: arithmetic of every projection below
  int kv16;  // key/value caches (accumulator, layers, temporal) stored in BF16
  QW in, acc_q, acc_kv, acc_o, head1, head2;
  float* calib = nullptr;  // calibration: per-input maxima (FP32 models only)
  CtWeights ct{};          // channel groups only
};

// Projection inputs, in calibration-slot order: latent embedding,
// accumulator q / kv / o, per layer QKV, O, gate/up (one input), down, then
// head W1 and W2.
__host__ __device__ inline int act_points(int L) { return 6 + 4 * L; }

struct NetDims {
  int L, d, heads, dh, r, s, F, C, Ch, n_acc, n_sp, n_tm;
  int cycle;  // 0: wavefront schedule; c: cyclic schedule of c steps
  float ln_smin, ln_smax, inv_delta;
  // Channel Transformer: groups (0: plain head), width, per-group width,
  // channels per group, per-group SwiGLU width, blocks
  int cg, cd, cdg, cCg, cFg, cL;
};

// Buffers and row maps of one pass.
struct PassCtx {
  int M;
  const int* gpos;            // global position of each row (null: identity)
  const int* fid;             // frame of each row (null: frame0)
  const FrameInfo* frames;
  FrameInfo frame0;
  int HWt;
  const float* h;             // hyper tokens [HWt][d]
  float* acc_kv;              // [HWt][2d]
  float* kv;                  // layer 0 K/V [HWt][2d]; layer l at kv + l * kv_stride
  size_t kv_stride;
  const float* tkv;           // layer 0 temporal K/V [2][HWt][2d] (or null)
  size_t tkv_stride;
  float *x, *q, *att, *e, *t1, *hmid;  // row activations
  float *ct_c, *ct_u, *ct_h, *ct_t1;   // Channel Transformer rows: stream [M][cd], block
                                       // inputs [cL][.][cd], SwiGLU [M][cFg], head [M][cdg]
  size_t ct_u_stride;                  // floats between ct_u's blocks (0: M * cd)
  float *mean, *scale, *bits;          // [HWt][C]
  int32_t* center;
  uint16_t* index;
  int32_t* center_c;          // compact copies for the bitstream decoder (or null)
  uint16_t* index_c;
  int* flag;
  const int32_t* ysrc;        // symbol source
  int src_compact;            // 1: ysrc is [M][C] compact, 0: [HWt][C]
  int32_t* ydec;              // decoded symbols [HWt][C]
};

struct NetOp {
  int kind;      // 0: GEMM, 1: attention, 2: symbols (gather + bits)
  int ak, rms, epi;
};

__host__ __device__ inline GemmArgs gemm_base(int M, int N, int K, int role) {
  GemmArgs g{};
  g.M = M;
  g.N = N;
  g.K = K;
  g.role = role;
  return g;
}

__host__ __device__ inline void use_q(GemmArgs& g, const DevWeights& dw, QW w, QW w2 = QW{},
                                     size_t off = 0, size_t off2 = 0) {
  if (dw.calib && w.slot >= 0) g.amax = dw.calib + w.slot;
  const int prec = dw.prec;
  if (prec == 0 || !w.q) return;
  const int eb = prec == 1 ? 2 : 1;
  g.prec = prec;
  g.Wq = static_cast<const char*>(w.q) + off * eb;
  g.wscale = w.inv_scale;
  g.ascale = w.ascale;
  if (w2.q) {
    g.W2q = static_cast<const char*>(w2.q) + off2 * eb;
    g.w2scale = w2.inv_scale;
  }
}

__host__ __device__ inline AttnArgs attn_base(const NetDims& x, const PassCtx& c, int role) {
  AttnArgs a{};
  a.role = role;
  a.M = c.M;
  a.pos = c.gpos;
  a.fid = c.fid;
  a.frames = c.frames;
  a.frame0 = c.frame0;
  a.HWt = c.HWt;
  a.r = x.r;
  a.cycle = x.cycle;
  a.heads = x.heads;
  a.dh = x.dh;
  a.d = x.d;
  a.q = c.q;
  a.ldq = x.d;
  a.out = c.att;
  a.ldo = x.d;
  return a;
}

// ---- accumulator
__host__ __device__ inline GemmArgs args_acc_q(const NetDims& x, const DevWeights& w,
                                               const PassCtx& c) {
  GemmArgs g = gemm_base(c.M, x.d, x.d, R_ACC_Q);
  g.X = c.h; g.ldx = x.d; g.xrow = c.gpos; g.gain = w.acc_gq; g.W = w.acc_Wq;
  g.Y = c.q; g.ldy = x.d;
  use_q(g, w, w.acc_q);
  return g;
}
__host__ __device__ inline AttnArgs args_acc_attn(const NetDims& x, const DevWeights& w,
                                                  const PassCtx& c) {
  AttnArgs a = attn_base(x, c, R_ACC_ATTN);
  a.kv = c.acc_kv; a.tkv = nullptr; a.kv16 = w.kv16; a.bias = w.acc_bias; a.nbias = x.n_acc;
  a.knull = w.knull; a.vnull = w.vnull; a.include_self = 0;
  return a;
}
__host__ __device__ inline GemmArgs args_acc_o(const NetDims& x, const DevWeights& w,
                                               const PassCtx& c) {
  GemmArgs g = gemm_base(c.M, x.d, x.d, R_ACC_O);
  g.X = c.att; g.ldx = x.d; g.W = w.acc_Wo;
  g.R = c.h; g.ldr = x.d; g.rrow = c.gpos; g.Y = c.x; g.ldy = x.d;
  use_q(g, w, w.acc_o);
  return g;
}

// ---- layers
__host__ __device__ inline GemmArgs args_qkv(const NetDims& x, const DevWeights& w,
                                             const PassCtx& c, int l) {
  const LayerWeights& L = w.layers[l];
  GemmArgs g = gemm_base(c.M, 3 * x.d, x.d, R_QKV);
  g.X = c.x; g.ldx = x.d; g.gain = L.g1; g.W = L.Wqkv;
  g.Y = c.q; g.ldy = x.d; g.Y2 = c.kv + l * c.kv_stride; g.ldy2 = 2 * x.d; g.y2row = c.gpos;
  g.nsplit = x.d;
  g.kv16 = w.kv16;
  use_q(g, w, L.qkv);
  return g;
}
__host__ __device__ inline AttnArgs args_attn(const NetDims& x, const DevWeights& w,
                                              const PassCtx& c, int l) {
  AttnArgs a = attn_base(x, c, R_ATTN);
  a.kv = c.kv + l * c.kv_stride;
  a.tkv = c.tkv ? c.tkv + l * c.tkv_stride : nullptr;
  a.kv16 = w.kv16;
  a.bias = w.layers[l].bias; a.nbias = x.n_sp + x.n_tm;
  a.knull = nullptr; a.vnull = nullptr; a.include_self = 1;
  return a;
}
__host__ __device__ inline GemmArgs args_o(const NetDims& x, const DevWeights& w,
                                           const PassCtx& c, int l) {
  GemmArgs g = gemm_base(c.M, x.d, x.d, R_O);
  g.X = c.att; g.ldx = x.d; g.W = w.layers[l].Wo;
  g.R = c.x; g.ldr = x.d; g.Y = c.x; g.ldy = x.d;
  use_q(g, w, w.layers[l].o);
  return g;
}
__host__ __device__ inline GemmArgs args_gateup(const NetDims& x, const DevWeights& w,
                                                const PassCtx& c, int l) {
  GemmArgs g = gemm_base(c.M, x.F, x.d, R_GATEUP);
  g.X = c.x; g.ldx = x.d; g.gain = w.layers[l].g2; g.W = w.layers[l].Wgate;
  g.W2 = w.layers[l].Wup; g.Y = c.hmid; g.ldy = x.F;
  use_q(g, w, w.layers[l].gate, w.layers[l].up);
  return g;
}
__host__ __device__ inline GemmArgs args_down(const NetDims& x, const DevWeights& w,
                                              const PassCtx& c, int l) {
  GemmArgs g = gemm_base(c.M, x.d, x.F, R_DOWN);
  g.X = c.hmid; g.ldx = x.F; g.W = w.layers[l].Wdown;
  g.R = c.x; g.ldr = x.d; g.Y = c.x; g.ldy = x.d;
  use_q(g, w, w.layers[l].down);
  return g;
}

// ---- head
__host__ __device__ inline GemmArgs args_head1(const NetDims& x, const DevWeights& w,
                                               const PassCtx& c) {
  GemmArgs g = gemm_base(c.M, x.d, x.d, R_HEAD1);
  g.X = c.x; g.ldx = x.d; g.gain = w.head_g; g.W = w.W1; g.Y = c.t1; g.ldy = x.d;
  use_q(g, w, w.head1);
  return g;
}
__host__ __device__ inline GemmArgs args_head2(const NetDims& x, const DevWeights& w,
                                               const PassCtx& c) {
  GemmArgs g = gemm_base(c.M, x.C, x.d, R_HEAD2);
  g.X = c.t1; g.ldx = x.d; g.W = w.W2; g.W2 = w.W2 + (size_t)x.C * x.d; g.yrow = c.gpos;
  g.head.gmu = w.gmu; g.head.bmu = w.bmu; g.head.gsig = w.gsig; g.head.bsig = w.bsig;
  g.head.ln_smin = x.ln_smin; g.head.ln_smax = x.ln_smax; g.head.inv_delta = x.inv_delta;
  g.head.ldo = x.C; g.head.col0 = 0;
  g.head.mean = c.mean; g.head.scale = c.scale; g.head.center = c.center;
  g.head.index = c.index; g.head.center_c = c.center_c; g.head.index_c = c.index_c;
  g.head.flag = c.flag;
  use_q(g, w, w.head2, w.head2, 0, (size_t)x.C * x.d);
  return g;
}

// ---- Channel Transformer, channel group g (each GEMM on the group's slice
// of the [M][cd] stream; the rows' positions index ydec)
__host__ __device__ inline GemmArgs args_ct_in(const NetDims& x, const DevWeights& w,
                                               const PassCtx& c, int g) {
  GemmArgs a = gemm_base(c.M, x.cdg, x.d, R_HEAD1);
  a.X = c.x; a.ldx = x.d; a.gain = w.ct.gx; a.W = w.ct.Wx + (size_t)g * x.cdg * x.d;
  a.Y = c.ct_c + (size_t)g * x.cdg; a.ldy = x.cd;
  return a;
}
__host__ __device__ inline GemmArgs args_ct_latent(const NetDims& x, const DevWeights& w,
                                                   const PassCtx& c, int g) {
  GemmArgs a = gemm_base(c.M, x.cdg, g * x.cCg, R_HEAD1);
  a.Xi = c.ydec; a.ldx = x.C; a.xrow = c.gpos; a.xscale = w.ct.gy; a.W = w.ct.wy_g[g];
  a.R = c.ct_c + (size_t)g * x.cdg; a.ldr = x.cd; a.Y = c.ct_c + (size_t)g * x.cdg; a.ldy = x.cd;
  return a;
}
// Block b's per-group normalized inputs.
__host__ __device__ inline float* ct_u_block(const NetDims& x, const PassCtx& c, int b) {
  return c.ct_u + (size_t)b * (c.ct_u_stride ? c.ct_u_stride : (size_t)c.M * x.cd);
}
// Block b's RMSNorm of group g's slice of the stream, as a row description:
// rows M, slice K = cdg at column col0 (in n), input X, gain, output Y.
__host__ __device__ inline GemmArgs args_ct_rms(const NetDims& x, const DevWeights& w,
                                                const PassCtx& c, int b, int g) {
  GemmArgs a = gemm_base(c.M, x.cdg, x.cdg, R_OTHER);
  a.X = c.ct_c; a.ldx = x.cd; a.gain = w.ct.g1[b]; a.Y = ct_u_block(x, c, b); a.ldy = x.cd;
  a.nsplit = g * x.cdg;  // the slice's first column
  return a;
}
__host__ __device__ inline GemmArgs args_ct_mix(const NetDims& x, const DevWeights& w,
                                                const PassCtx& c, int b, int g) {
  GemmArgs a = gemm_base(c.M, x.cdg, (g + 1) * x.cdg, R_HEAD1);
  a.X = ct_u_block(x, c, b); a.ldx = x.cd; a.W = w.ct.m_g[b][g];
  a.R = c.ct_c + (size_t)g * x.cdg; a.ldr = x.cd; a.Y = c.ct_c + (size_t)g * x.cdg; a.ldy = x.cd;
  return a;
}
__host__ __device__ inline GemmArgs args_ct_gateup(const NetDims& x, const DevWeights& w,
                                                   const PassCtx& c, int b, int g) {
  GemmArgs a = gemm_base(c.M, x.cFg, x.cdg, R_HEAD1);
  a.X = c.ct_c + (size_t)g * x.cdg; a.ldx = x.cd; a.gain = w.ct.g2[b] + (size_t)g * x.cdg;
  a.W = w.ct.Wgate[b] + (size_t)g * x.cFg * x.cdg; a.W2 = w.ct.Wup[b] + (size_t)g * x.cFg * x.cdg;
  a.Y = c.ct_h; a.ldy = x.cFg;
  return a;
}
__host__ __device__ inline GemmArgs args_ct_down(const NetDims& x, const DevWeights& w,
                                                 const PassCtx& c, int b, int g) {
  GemmArgs a = gemm_base(c.M, x.cdg, x.cFg, R_HEAD1);
  a.X = c.ct_h; a.ldx = x.cFg; a.W = w.ct.Wdown[b] + (size_t)g * x.cdg * x.cFg;
  a.R = c.ct_c + (size_t)g * x.cdg; a.ldr = x.cd; a.Y = c.ct_c + (size_t)g * x.cdg; a.ldy = x.cd;
  return a;
}
__host__ __device__ inline GemmArgs args_ct_head1(const NetDims& x, const DevWeights& w,
                                                  const PassCtx& c, int g) {
  GemmArgs a = gemm_base(c.M, x.cdg, x.cdg, R_HEAD1);
  a.X = c.ct_c + (size_t)g * x.cdg; a.ldx = x.cd; a.gain = w.ct.hg + (size_t)g * x.cdg;
  a.W = w.ct.W1 + (size_t)g * x.cdg * x.cdg; a.Y = c.ct_t1; a.ldy = x.cdg;
  return a;
}
__host__ __device__ inline GemmArgs args_ct_head2(const NetDims& x, const DevWeights& w,
                                                  const PassCtx& c, int g) {
  GemmArgs a = args_head2(x, w, c);
  const float* W2g = w.ct.W2 + (size_t)g * 2 * x.cCg * x.cdg;
  a.N = x.cCg; a.K = x.cdg;
  a.X = c.ct_t1; a.ldx = x.cdg; a.W = W2g; a.W2 = W2g + (size_t)x.cCg * x.cdg;
  a.prec = 0; a.Wq = nullptr; a.W2q = nullptr; a.wscale = a.w2scale = 1.f; a.ascale = 0.f;
  a.amax = nullptr;
  a.head.col0 = g * x.cCg;
  return a;
}

// ---- embedding of decoded symbols (rows read from ydec at their positions)
__host__ __device__ inline GemmArgs args_embed(const NetDims& x, const DevWeights& w,
                                               const PassCtx& c) {
  GemmArgs g = gemm_base(c.M, x.d, x.C, R_EMBED);
  g.Xi = c.ydec; g.ldx = x.C; g.xrow = c.gpos; g.xscale = w.ing; g.W = w.inW;
  g.Y = c.e; g.ldy = x.d;
  use_q(g, w, w.in);
  return g;
}
__host__ __device__ inline GemmArgs args_acc_kv(const NetDims& x, const DevWeights& w,
                                                const PassCtx& c) {
  GemmArgs g = gemm_base(c.M, 2 * x.d, x.d, R_ACCKV);
  g.X = c.e; g.ldx = x.d; g.gain = w.acc_gkv; g.W = w.acc_Wkv;
  g.Y = c.acc_kv; g.ldy = 2 * x.d; g.yrow = c.gpos; g.kv16 = w.kv16;
  use_q(g, w, w.acc_kv);
  return g;
}

}  // namespace pswa
