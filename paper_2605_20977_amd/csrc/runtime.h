// Host runtime pieces shared by the C ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/pswa.h"
#include "network.h"
#include "pswa_internal.h"

struct pswa_model {
  pswa_model_desc desc;
  pswa::NetDims x;
  pswa::DevWeights w;
};

namespace pswa {

pswa_status fail(pswa_status st, const char* fmt, ...);

#define PSWA_HIP_TRY(expr)                                                          \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return ::pswa::fail(PSWA_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Bump allocator over a caller-provided region (also used to size it).
struct Layout {
  char* base;
  size_t used = 0;
  explicit Layout(void* b = nullptr) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    T* p = base ? reinterpret_cast<T*>(base + used) : nullptr;
    used += align_up(count * sizeof(T));
    return p;
  }
};

bool valid_frame(const pswa_frame_desc* f, std::string* why);
bool model_desc_valid(const pswa_model_desc* d, std::string* why);
NetDims model_dims(const pswa_model_desc& d);
// (offset, floats) of every tensor of the weight blob, in blob order, each
// tensor starting at a multiple of `align` floats; returns the total floats.
size_t model_blob_spans(const NetDims& x, size_t align,
                        std::vector<std::pair<size_t, size_t>>* spans);
// Decoding schedule of a model. Wavefront (cycle 0): step t holds the
// positions (i, t - s i), i ascending, s = r + 1, and a frame takes
// (W - 1) + s (H - 1) + 1 steps. Cyclic (cycle c): step t holds every
// (i, j) with (i + j) mod c = t, in raster order, and a frame takes c steps.
inline int sched_steps(const NetDims& x, int H, int W) {
  return x.cycle ? x.cycle : (W - 1) + x.s * (H - 1) + 1;
}
template <class F>
void sched_for_each(const NetDims& x, int H, int W, int t, F f) {
  if (x.cycle) {
    for (int i = 0; i < H; ++i)
      for (int j = ((t - i) % x.cycle + x.cycle) % x.cycle; j < W; j += x.cycle) f(i, j);
  } else {
    for (int i = 0; i < H; ++i) {
      const int j = t - x.s * i;
      if (j >= 0 && j < W) f(i, j);
    }
  }
}
inline int sched_len(const NetDims& x, int H, int W, int t) {
  int n = 0;
  sched_for_each(x, H, W, t, [&](int, int) { ++n; });
  return n;
}

// Row activations for `rows` rows (and the Channel Transformer's, if any).
struct Acts {
  float *x, *q, *att, *e, *t1, *hmid;
  float *ct_c, *ct_u, *ct_h, *ct_t1;
};
Acts take_acts(Layout& L, const NetDims& x, size_t rows);

// Channel group g of the Channel Transformer over c's rows: its input
// (spatial output, and the latent's groups 0 .. g-1 read from c.ydec at the
// rows' positions), the blocks (per-group RMSNorm, masked mixing over groups
// 0 .. g, per-group SwiGLU) and the group's head (mean, scale and CDF
// selection of its channels).
inline void run_ct_group(const pswa_model* m, const PassCtx& c, int g, hipStream_t st) {
  const NetDims& x = m->x;
  const DevWeights& w = m->w;
  gemm_run(A_FLOAT, true, EPI_STORE, args_ct_in(x, w, c, g), st);
  if (g > 0) gemm_run(A_INT, false, EPI_RESID, args_ct_latent(x, w, c, g), st);
  for (int b = 0; b < x.cL; ++b) {
    group_rmsnorm(c.ct_c, x.cd, c.M, x.cdg, g * x.cdg, w.ct.g1[b], ct_u_block(x, c, b), x.cd, st);
    gemm_run(A_FLOAT, false, EPI_RESID, args_ct_mix(x, w, c, b, g), st);
    gemm_run(A_FLOAT, true, EPI_SWIGLU, args_ct_gateup(x, w, c, b, g), st);
    gemm_run(A_FLOAT, false, EPI_RESID, args_ct_down(x, w, c, b, g), st);
  }
  gemm_run(A_FLOAT, true, EPI_SILU, args_ct_head1(x, w, c, g), st);
  gemm_run(A_FLOAT, false, EPI_HEAD, args_ct_head2(x, w, c, g), st);
}

// One pass of the network over c's rows with per-phase launches.
// before_layer(l) runs before layer l's QKV (the encode form builds the
// layer's temporal K/V there); after_group(g) runs after channel group g's
// prediction (a decoder reads the group's symbols there; models without
// channel groups call it once, g = 0).
template <class BeforeLayer, class AfterGroup>
void run_pass(const pswa_model* m, const PassCtx& c, BeforeLayer before_layer,
              AfterGroup after_group, hipStream_t st) {
  const NetDims& x = m->x;
  const DevWeights& w = m->w;
  gemm_run(A_FLOAT, true, EPI_STORE, args_acc_q(x, w, c), st);
  attention_f32(args_acc_attn(x, w, c), st);
  gemm_run(A_FLOAT, false, EPI_RESID, args_acc_o(x, w, c), st);
  for (int l = 0; l < x.L; ++l) {
    before_layer(l);
    gemm_run(A_FLOAT, true, EPI_QKV, args_qkv(x, w, c, l), st);
    attention_f32(args_attn(x, w, c, l), st);
    gemm_run(A_FLOAT, false, EPI_RESID, args_o(x, w, c, l), st);
    gemm_run(A_FLOAT, true, EPI_SWIGLU, args_gateup(x, w, c, l), st);
    gemm_run(A_FLOAT, false, EPI_RESID, args_down(x, w, c, l), st);
  }
  if (x.cg) {
    for (int g = 0; g < x.cg; ++g) {
      run_ct_group(m, c, g, st);
      after_group(g);
    }
    return;
  }
  gemm_run(A_FLOAT, true, EPI_SILU, args_head1(x, w, c), st);
  gemm_run(A_FLOAT, false, EPI_HEAD, args_head2(x, w, c), st);
  after_group(0);
}

// Embedding of decoded symbols (read from c.ydec at the rows' positions) and
// their accumulator K/V.
void run_embed(const pswa_model* m, const PassCtx& c, hipStream_t st);

// e_prev[tau] (rows off .. off+HW of a [2][HWt][d] buffer) from prev [2][HW][C].
void embed_prev(const pswa_model* m, int HW, int HWt, int off, const int32_t* prev, float* e_prev,
                hipStream_t st);
// Layer-l temporal K/V (rows off .. off+HW of [2][HWt][2d]) from e_prev.
void temporal_kv_layer(const pswa_model* m, int HW, int HWt, int off, const float* e_prev, int l,
                       float* tkv_l, hipStream_t st);

// The parallel encode form with its workspace at d_ws (the body of
// pswa_encode_params; the no-allocation variant passes its static scratch).
pswa_status encode_into(const pswa_model* model, const pswa_frame_desc* frame,
                        const int32_t* d_latents, const int32_t* d_hyper, const int32_t* d_prev,
                        float* d_mean, float* d_scale, float* d_bits, int32_t* d_cdf_center,
                        uint16_t* d_cdf_index, double* h_total_bits, void* d_ws, size_t ws_bytes,
                        void* stream);

pswa_status finish_sum(const float* bits, size_t n, float* d_sum, const int* d_flag,
                       double* h_total, hipStream_t st);

}  // namespace pswa
