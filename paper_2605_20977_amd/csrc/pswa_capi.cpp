// C ABI and host runtime of the wavefront context model (see include/pswa.h):
// model upload, the parallel encode form, the per-diagonal decode and the
// entropy-coder calls.
//
// The runtime owns no device memory: it lays out caller-provided regions
// (model weights, encode workspace, decode state) and enqueues kernels on the
// caller's stream. The same row-wise kernels run the parallel encode form
// (all H*W positions per launch) and the decode steps (the n_t positions of
// one diagonal per launch).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/pswa.h"
#include "persistent.h"
#include "runtime.h"

using namespace pswa;

namespace pswa {

namespace {
thread_local std::string g_last_error;
}  // namespace

pswa_status fail(pswa_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

const char* last_error() { return g_last_error.c_str(); }

bool valid_frame(const pswa_frame_desc* f, std::string* why) {
  if (!f) return *why = "null frame desc", false;
  if (f->H < 1 || f->W < 1 || (int64_t)f->H * f->W > (1 << 24))
    return *why = "H, W must be >= 1 with H*W <= 2^24", false;
  if (f->Hh != (f->H + 3) / 4 || f->Wh != (f->W + 3) / 4)
    return *why = "hyperprior grid must be ceil(H/4) x ceil(W/4)", false;
  if (f->n_prev != 0 && f->n_prev != 2) return *why = "n_prev must be 0 or 2", false;
  return true;
}


Acts take_acts(Layout& L, const NetDims& x, size_t rows) {
  Acts a;
  a.x = L.take<float>(rows * x.d);
  a.q = L.take<float>(rows * x.d);
  a.att = L.take<float>(rows * x.d);
  a.e = L.take<float>(rows * x.d);
  a.t1 = L.take<float>(rows * x.d);
  a.hmid = L.take<float>(rows * x.F);
  a.ct_c = a.ct_u = a.ct_h = a.ct_t1 = nullptr;
  if (x.cg) {
    a.ct_c = L.take<float>(rows * x.cd);
    a.ct_u = L.take<float>((size_t)x.cL * rows * x.cd);
    a.ct_h = L.take<float>(rows * x.cFg);
    a.ct_t1 = L.take<float>(rows * x.cdg);
  }
  return a;
}

void run_embed(const pswa_model* m, const PassCtx& c, hipStream_t st) {
  gemm_run(A_INT, false, EPI_STORE, args_embed(m->x, m->w, c), st);
  gemm_run(A_FLOAT, true, EPI_STORE, args_acc_kv(m->x, m->w, c), st);
}

void embed_prev(const pswa_model* m, int HW, int HWt, int off, const int32_t* prev, float* e_prev,
                hipStream_t st) {
  const NetDims& x = m->x;
  for (int tau = 0; tau < 2; ++tau) {
    GemmArgs a = gemm_base(HW, x.d, x.C, R_TKV);
    a.Xi = prev + (size_t)tau * HW * x.C; a.ldx = x.C; a.xscale = m->w.ing; a.W = m->w.inW;
    a.Y = e_prev + ((size_t)tau * HWt + off) * x.d; a.ldy = x.d;
    use_q(a, m->w, m->w.in);
    gemm_run(A_INT, false, EPI_STORE, a, st);
  }
}

void temporal_kv_layer(const pswa_model* m, int HW, int HWt, int off, const float* e_prev, int l,
                       float* tkv_l, hipStream_t st) {
  const NetDims& x = m->x;
  for (int tau = 0; tau < 2; ++tau) {
    GemmArgs a = gemm_base(HW, 2 * x.d, x.d, R_TKV);
    a.X = e_prev + ((size_t)tau * HWt + off) * x.d; a.ldx = x.d; a.gain = m->w.layers[l].g1;
    a.W = m->w.layers[l].Wqkv + (size_t)x.d * x.d;
    const size_t e0 = ((size_t)tau * HWt + off) * 2 * x.d;  // element offset of the rows
    a.Y = m->w.kv16 ? reinterpret_cast<float*>(reinterpret_cast<uint16_t*>(tkv_l) + e0)
                    : tkv_l + e0;
    a.ldy = 2 * x.d;
    a.kv16 = m->w.kv16;
    use_q(a, m->w, m->w.layers[l].qkv, QW{}, (size_t)x.d * x.d);
    gemm_run(A_FLOAT, true, EPI_STORE, a, st);
  }
}

pswa_status finish_sum(const float* bits, size_t n, float* d_sum, const int* d_flag,
                       double* h_total, hipStream_t st) {
  sum_f32(bits, n, d_sum, st);
  PSWA_HIP_TRY(hipGetLastError());
  float s = 0.f;
  int flag = 0;
  PSWA_HIP_TRY(hipMemcpyAsync(&s, d_sum, sizeof s, hipMemcpyDeviceToHost, st));
  PSWA_HIP_TRY(hipMemcpyAsync(&flag, d_flag, sizeof flag, hipMemcpyDeviceToHost, st));
  PSWA_HIP_TRY(hipStreamSynchronize(st));
  *h_total = double(s);
  if (flag) return fail(PSWA_E_NUMERIC, "non-finite mean or scale produced");
  return PSWA_OK;
}

}  // namespace pswa

namespace {

constexpr size_t kTensorAlign = 64;  // floats

bool valid_desc(const pswa_model_desc* d, std::string* why) {
  if (!d) return *why = "null model desc", false;
  if (d->L < 1 || d->L > kMaxLayers) return *why = "L out of range [1, 16]", false;
  if (d->d < 64 || d->d % 64 != 0 || d->d > 1024) return *why = "d must be a multiple of 64 in [64, 1024]", false;
  if (d->heads < 1 || d->d % d->heads != 0) return *why = "heads must divide d", false;
  const int dh = d->d / d->heads;
  if (dh != 16 && dh != 32 && dh != 48 && dh != 64) return *why = "head dim must be 16, 32, 48 or 64", false;
  if (d->window < 3 || d->window > 9 || d->window % 2 == 0) return *why = "window must be odd in [3, 9]", false;
  if (d->mlp_ratio < 1 || d->mlp_ratio * d->d > 2048) return *why = "mlp_ratio * d must be in [d, 2048]", false;
  if (d->C < 4 || d->C > 256 || d->C % 4 != 0) return *why = "C must be a multiple of 4 in [4, 256]", false;
  if (d->Ch < 1 || d->Ch > 512) return *why = "Ch out of range [1, 512]", false;
  if (d->prec != PSWA_FP32 && d->prec != PSWA_BF16 && d->prec != PSWA_FP8_E4M3)
    return *why = "unknown precision", false;
  if (d->cycle != 0 && (d->cycle < 2 || d->cycle > 16))
    return *why = "cycle must be 0 (wavefront) or in [2, 16]", false;
  if (d->act_scaling != PSWA_ACT_TENSOR &&
      !(d->prec == PSWA_FP8_E4M3 && d->act_scaling == PSWA_ACT_ROW))
    return *why = "act_scaling must be PSWA_ACT_TENSOR, or PSWA_ACT_ROW for FP8 models", false;
  if (d->ch_groups == 0) {
    if (d->ch_d != 0 || d->ch_L != 0)
      return *why = "ch_d and ch_L must be 0 without channel groups", false;
  } else {
    const int N = d->ch_groups;
    if (N < 1 || N > kMaxChGroups) return *why = "ch_groups must be in [1, 8]", false;
    if (d->C % N != 0 || (d->C / N) % 4 != 0)
      return *why = "C / ch_groups must be a multiple of 4", false;
    if (d->ch_d % N != 0 || d->ch_d / N < 16 || d->ch_d / N > 512 || (d->ch_d / N) % 16 != 0)
      return *why = "ch_d / ch_groups must be a multiple of 16 in [16, 512]", false;
    if (d->ch_L < 1 || d->ch_L > kMaxChBlocks) return *why = "ch_L must be in [1, 4]", false;
    if (d->ch_ratio < 1 || d->ch_ratio > 4) return *why = "ch_ratio must be in [1, 4]", false;
  }
  return true;
}

// Whether the blob carries calibrated activation maxima after the weights.
bool has_act_maxima(const pswa_model_desc& d) {
  return d.prec == PSWA_FP8_E4M3 && d.act_scaling == PSWA_ACT_TENSOR;
}

NetDims dims_of(const pswa_model_desc& m) {
  NetDims x{};
  x.L = m.L;
  x.d = m.d;
  x.heads = m.heads;
  x.dh = m.d / m.heads;
  x.r = (m.window - 1) / 2;
  x.cycle = m.cycle;
  x.s = m.cycle ? m.cycle : x.r + 1;
  x.F = m.mlp_ratio * m.d;
  x.C = m.C;
  x.Ch = m.Ch;
  const int k2 = (2 * x.r + 1) * (2 * x.r + 1);
  x.n_acc = m.cycle ? k2 : 2 * x.r * (x.r + 1);
  x.n_sp = m.cycle ? k2 : x.n_acc + 1;
  x.n_tm = 2 * k2;
  x.ln_smin = ln_sigma_min_f32();
  x.ln_smax = float(std::log(kSigmaMax));
  x.inv_delta = inv_delta_f32();
  x.cg = m.ch_groups;
  if (x.cg) {
    x.cd = m.ch_d;
    x.cdg = m.ch_d / m.ch_groups;
    x.cCg = m.C / m.ch_groups;
    x.cFg = m.ch_ratio * x.cdg;
    x.cL = m.ch_L;
  }
  return x;
}

// Walks the documented blob order; with base == nullptr it only counts.
// align > 1 pads every tensor to a multiple of `align` floats (the device
// layout keeps each tensor 256-byte aligned for vector loads).
size_t blob_layout(const NetDims& x, const float* base, DevWeights* w, size_t align = 1,
                   std::vector<std::pair<size_t, size_t>>* spans = nullptr) {
  size_t off = 0;
  auto t = [&](size_t n) {
    const float* p = base ? base + off : nullptr;
    if (spans) spans->emplace_back(off, n);
    off += (n + align - 1) / align * align;
    return p;
  };
  const size_t d = x.d, C = x.C, Ch = x.Ch, F = x.F, h = x.heads;
  DevWeights tmp{};
  DevWeights& W = w ? *w : tmp;
  W.hyperW = t(d * Ch);
  W.P4 = t(16 * d);
  W.ing = t(C);
  W.inW = t(d * C);
  W.acc_gq = t(d);
  W.acc_Wq = t(d * d);
  W.acc_gkv = t(d);
  W.acc_Wkv = t(2 * d * d);
  W.knull = t(d);
  W.vnull = t(d);
  W.acc_bias = t(h * x.n_acc);
  W.acc_Wo = t(d * d);
  for (int l = 0; l < x.L; ++l) {
    LayerWeights& L = W.layers[l];
    L.g1 = t(d);
    L.Wqkv = t(3 * d * d);
    L.bias = t(h * (x.n_sp + x.n_tm));
    L.Wo = t(d * d);
    L.g2 = t(d);
    L.Wgate = t(F * d);
    L.Wup = t(F * d);
    L.Wdown = t(d * F);
  }
  if (x.cg) {  // Channel Transformer in place of the plain head
    const size_t N = x.cg, dc = x.cd, dg = x.cdg, Cg = x.cCg, Fg = x.cFg;
    CtWeights& T = W.ct;
    T.gx = t(d);
    T.Wx = t(dc * d);
    T.gy = t(C);
    T.Wy = t(dc * C);
    for (int b = 0; b < x.cL; ++b) {
      T.g1[b] = t(dc);
      T.M[b] = t(dc * dc);
      T.g2[b] = t(dc);
      T.Wgate[b] = t(N * Fg * dg);
      T.Wup[b] = t(N * Fg * dg);
      T.Wdown[b] = t(N * dg * Fg);
    }
    T.hg = t(dc);
    T.W1 = t(N * dg * dg);
    T.W2 = t(N * 2 * Cg * dg);
    W.head_g = W.W1 = W.W2 = nullptr;
  } else {
    W.head_g = t(d);
    W.W1 = t(d * d);
    W.W2 = t(2 * C * d);
  }
  W.gmu = t(C);
  W.bmu = t(C);
  W.gsig = t(C);
  W.bsig = t(C);
  return off;
}

// Projection weights that run in the model's GEMM precision: tensor index in
// the blob order, field of DevWeights that receives the copy, and the
// weight's K (its row length).
struct QuantTarget {
  int tensor;
  QW* dst;
  int K;
};
// Calibration slot of every projection input (see act_points): gate and up
// share their input.
void assign_slots(DevWeights& w, const NetDims& x) {
  w.in.slot = 0;
  w.acc_q.slot = 1;
  w.acc_kv.slot = 2;
  w.acc_o.slot = 3;
  for (int l = 0; l < x.L; ++l) {
    LayerWeights& Ly = w.layers[l];
    Ly.qkv.slot = 4 + 4 * l;
    Ly.o.slot = 5 + 4 * l;
    Ly.gate.slot = Ly.up.slot = 6 + 4 * l;
    Ly.down.slot = 7 + 4 * l;
  }
  w.head1.slot = 4 + 4 * x.L;
  w.head2.slot = 5 + 4 * x.L;
}

std::vector<QuantTarget> quant_targets(DevWeights& w, const NetDims& x) {
  std::vector<QuantTarget> t = {
      {3, &w.in, x.C}, {5, &w.acc_q, x.d}, {7, &w.acc_kv, x.d}, {11, &w.acc_o, x.d}};
  for (int l = 0; l < x.L; ++l) {
    LayerWeights& Ly = w.layers[l];
    t.push_back({13 + 8 * l, &Ly.qkv, x.d});
    t.push_back({15 + 8 * l, &Ly.o, x.d});
    t.push_back({17 + 8 * l, &Ly.gate, x.d});
    t.push_back({18 + 8 * l, &Ly.up, x.d});
    t.push_back({19 + 8 * l, &Ly.down, x.F});
  }
  if (!x.cg) {  // (the Channel Transformer runs in FP32)
    t.push_back({13 + 8 * x.L, &w.head1, x.d});
    t.push_back({14 + 8 * x.L, &w.head2, x.d});
  }
  return t;
}

// Row-major [N][K] low-precision weight (eb bytes per element) to the MFMA
// fragment layout: units of 8 rows, k-step blocks of 32 columns, chunk
// (8 * kg + row % 8) of 8 consecutive values per block. Needs N % 8 == 0
// and K % 32 == 0.
std::vector<uint8_t> to_fragment_layout(const std::vector<uint8_t>& rm, size_t N, size_t K,
                                        size_t eb) {
  std::vector<uint8_t> out(rm.size());
  const size_t ks = K / 32;
  for (size_t n = 0; n < N; ++n)
    for (size_t k = 0; k < K; k += 8) {
      const size_t chunk = 8 * ((k % 32) / 8) + n % 8;
      const size_t e = (((n / 8) * ks + k / 32) * 32 + chunk) * 8;
      std::memcpy(&out[e * eb], &rm[(n * K + k) * eb], 8 * eb);
    }
  return out;
}

uint16_t bf16_rne_host(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

// OCP FP8 e4m3fn (bias 7, 3 mantissa bits, max 448, no infinities), round
// to nearest even, saturating.
uint8_t fp8_e4m3_rne_host(float f) {
  const uint8_t sign = std::signbit(f) ? 0x80 : 0x00;
  const double a = std::fabs(double(f));
  if (!(a == a)) return 0x7f;
  if (a >= 448.0) return sign | 0x7e;
  if (a == 0.0) return sign;
  int e;
  std::frexp(a, &e);        // a = fr * 2^e, fr in [0.5, 1)
  int ex = e - 1;           // a = 1.m * 2^ex
  if (ex < -6) {            // subnormal: multiples of 2^-9
    const double q = std::nearbyint(a * 512.0);  // ties to even
    if (q >= 8.0) return sign | 0x08;            // rounds up to the smallest normal
    return sign | uint8_t(q);
  }
  double q = std::nearbyint((a / std::ldexp(1.0, ex) - 1.0) * 8.0);
  if (q >= 8.0) {
    q = 0.0;
    ++ex;
  }
  if (ex > 8 || (ex == 8 && q > 6.0)) return sign | 0x7e;
  return sign | uint8_t(((ex + 7) << 3) | int(q));
}

// ------------------------------------------------------------ encode ws
struct EncodeWs {
  float *h, *acc_kv, *kv, *tkv, *e_prev;
  Acts a;
  int* flag;
  float* sum;
  size_t bytes;
};

EncodeWs plan_encode(const NetDims& x, const pswa_frame_desc& f, void* base) {
  Layout L(base);
  const size_t HW = (size_t)f.H * f.W;
  EncodeWs w;
  w.h = L.take<float>(HW * x.d);
  w.acc_kv = L.take<float>((HW + 1) * 2 * x.d);  // + the null row
  w.kv = L.take<float>(HW * 2 * x.d);
  w.tkv = f.n_prev ? L.take<float>(2 * HW * 2 * x.d) : nullptr;
  w.e_prev = f.n_prev ? L.take<float>(2 * HW * x.d) : nullptr;
  w.a = take_acts(L, x, HW);
  w.flag = L.take<int>(64);
  w.sum = L.take<float>(64);
  w.bytes = L.used;
  return w;
}

}  // namespace

namespace pswa {
bool model_desc_valid(const pswa_model_desc* d, std::string* why) { return valid_desc(d, why); }
NetDims model_dims(const pswa_model_desc& d) { return dims_of(d); }
size_t model_blob_spans(const NetDims& x, size_t align,
                        std::vector<std::pair<size_t, size_t>>* spans) {
  return blob_layout(x, nullptr, nullptr, align, spans);
}
}  // namespace pswa

// ------------------------------------------------------------ decode state
struct pswa_state {
  const pswa_model* model;
  pswa_frame_desc f;
  int T = 0, next_t = 0, nmax = 0;
  int source = PSWA_SRC_DEVICE;
  const int32_t* d_src = nullptr;
  std::vector<uint8_t> stream;
  std::unique_ptr<RangeDecoder> dec;
  std::vector<int> start;  // [T+1]
  // device
  float *h, *acc_kv, *kv, *tkv, *e_prev;
  int32_t* ydec;
  float *mean, *scale, *bits;
  int32_t* center;
  uint16_t* index;
  int* pos_all;
  Acts a;
  int32_t* cc;
  uint16_t* ci;
  int32_t* csym;
  int* flag;
  float* sum;
  size_t bytes;
  // pinned host staging (bitstream mode)
  int32_t* h_cc = nullptr;
  uint16_t* h_ci = nullptr;
  int32_t* h_sym = nullptr;
  ~pswa_state() {
    if (h_cc) (void)hipHostFree(h_cc);
    if (h_ci) (void)hipHostFree(h_ci);
    if (h_sym) (void)hipHostFree(h_sym);
  }
};

namespace {

void plan_state(const NetDims& x, const pswa_frame_desc& f, void* base, pswa_state* st) {
  Layout L(base);
  const size_t HW = (size_t)f.H * f.W;
  st->T = sched_steps(x, f.H, f.W);
  int nmax = 1;
  for (int t = 0; t < st->T; ++t) nmax = std::max(nmax, sched_len(x, f.H, f.W, t));
  st->nmax = nmax;
  st->h = L.take<float>(HW * x.d);
  st->acc_kv = L.take<float>((HW + 1) * 2 * x.d);  // + the null row
  st->kv = L.take<float>((size_t)x.L * HW * 2 * x.d);
  st->tkv = f.n_prev ? L.take<float>((size_t)x.L * 2 * HW * 2 * x.d) : nullptr;
  st->e_prev = f.n_prev ? L.take<float>(2 * HW * x.d) : nullptr;
  st->ydec = L.take<int32_t>(HW * x.C);
  st->mean = L.take<float>(HW * x.C);
  st->scale = L.take<float>(HW * x.C);
  st->bits = L.take<float>(HW * x.C);
  st->center = L.take<int32_t>(HW * x.C);
  st->index = L.take<uint16_t>(HW * x.C);
  st->pos_all = L.take<int>(HW);
  st->a = take_acts(L, x, nmax);
  st->cc = L.take<int32_t>((size_t)nmax * x.C);
  st->ci = L.take<uint16_t>((size_t)nmax * x.C);
  st->csym = L.take<int32_t>((size_t)nmax * x.C);
  st->flag = L.take<int>(64);
  st->sum = L.take<float>(64);
  st->bytes = L.used;
}

PassCtx frame_ctx(const pswa_frame_desc& f) {
  PassCtx c{};
  c.frame0 = FrameInfo{f.H, f.W, 0, f.n_prev};
  c.HWt = f.H * f.W;
  return c;
}

}  // namespace

extern "C" {

const char* pswa_last_error(void) { return pswa::last_error(); }

size_t pswa_model_blob_floats(const pswa_model_desc* desc) {
  std::string why;
  if (!valid_desc(desc, &why)) return 0;
  const NetDims x = dims_of(*desc);
  return blob_layout(x, nullptr, nullptr) + (has_act_maxima(*desc) ? act_points(x.L) : 0);
}

int pswa_act_points(const pswa_model_desc* desc) {
  std::string why;
  if (!valid_desc(desc, &why)) return 0;
  return act_points(desc->L);
}

// Device layout: the FP32 weights (each tensor 256-byte aligned), then for
// BF16 / FP8 models a low-precision copy of every projection weight.
// Per-group compacted copies of the Channel Transformer's masked maps (FP32),
// placed from byte `at`: wy[g] ([dg][g Cg], g >= 1) and m[b * N + g]
// ([dg][(g + 1) dg]). Returns the end.
size_t ct_layout(const NetDims& x, size_t at, std::vector<size_t>* wy, std::vector<size_t>* m) {
  if (!x.cg) return at;
  for (int g = 0; g < x.cg; ++g) {
    if (wy) wy->push_back(at);
    at += align_up((size_t)x.cdg * g * x.cCg * sizeof(float));
  }
  for (int b = 0; b < x.cL; ++b)
    for (int g = 0; g < x.cg; ++g) {
      if (m) m->push_back(at);
      at += align_up((size_t)x.cdg * (g + 1) * x.cdg * sizeof(float));
    }
  return at;
}

size_t device_layout(const pswa_model_desc& desc, std::vector<std::pair<int, size_t>>* qoff,
                     std::vector<size_t>* ct_wy = nullptr, std::vector<size_t>* ct_m = nullptr) {
  const NetDims x = dims_of(desc);
  std::vector<std::pair<size_t, size_t>> spans;
  size_t bytes = align_up(blob_layout(x, nullptr, nullptr, kTensorAlign, &spans) * sizeof(float));
  if (desc.prec != PSWA_FP32) {
    const size_t eb = desc.prec == PSWA_BF16 ? 2 : 1;
    DevWeights tmp{};
    for (auto& t : quant_targets(tmp, x)) {
      if (qoff) qoff->push_back({t.tensor, bytes});
      bytes += align_up(spans[t.tensor].second * eb);
    }
  }
  return ct_layout(x, bytes, ct_wy, ct_m);
}

size_t pswa_model_device_bytes(const pswa_model_desc* desc) {
  std::string why;
  if (!valid_desc(desc, &why)) return 0;
  return device_layout(*desc, nullptr);
}

pswa_status pswa_model_create(const pswa_model_desc* desc, const float* h_blob,
                              size_t blob_floats, void* d_mem, size_t d_bytes, void* stream,
                              pswa_model** out) {
  std::string why;
  if (!out) return fail(PSWA_E_ARG, "out is null");
  *out = nullptr;
  if (!valid_desc(desc, &why)) return fail(PSWA_E_ARG, "invalid model desc: %s", why.c_str());
  if (!h_blob || !d_mem) return fail(PSWA_E_ARG, "null blob or device memory");
  if ((reinterpret_cast<uintptr_t>(d_mem) % kAlign) != 0)
    return fail(PSWA_E_ARG, "device memory must be 256-byte aligned");
  const NetDims x = dims_of(*desc);
  const size_t nweights = blob_layout(x, nullptr, nullptr);
  const size_t need = pswa_model_blob_floats(desc);
  if (blob_floats != need)
    return fail(PSWA_E_SHAPE, "blob has %zu floats, model needs %zu", blob_floats, need);
  if (has_act_maxima(*desc))
    for (int k = 0; k < act_points(x.L); ++k) {
      const float v = h_blob[nweights + k];
      if (!(v >= 0.f) || !std::isfinite(v))
        return fail(PSWA_E_ARG, "activation maximum %d is %g (must be finite and >= 0)", k, v);
    }
  if (d_bytes < pswa_model_device_bytes(desc))
    return fail(PSWA_E_ARG, "device region %zu bytes < %zu", d_bytes, pswa_model_device_bytes(desc));
  if (desc->prec != PSWA_FP32 && (x.C % 32 != 0 || x.d % 32 != 0))
    return fail(PSWA_E_UNSUPPORTED, "BF16/FP8 models need C and d multiples of 32");
  hipStream_t st = static_cast<hipStream_t>(stream);
  // Re-lay the blob with every tensor 256-byte aligned, then one upload.
  std::vector<std::pair<size_t, size_t>> src, dst;
  blob_layout(x, nullptr, nullptr, 1, &src);
  const size_t dev_floats = blob_layout(x, nullptr, nullptr, kTensorAlign, &dst);
  std::vector<float> padded(dev_floats, 0.f);
  for (size_t i = 0; i < src.size(); ++i)
    std::memcpy(padded.data() + dst[i].first, h_blob + src[i].first, src[i].second * sizeof(float));
  PSWA_HIP_TRY(hipMemcpyAsync(d_mem, padded.data(), dev_floats * sizeof(float),
                              hipMemcpyHostToDevice, st));
  std::unique_ptr<pswa_model> m(new pswa_model);
  m->desc = *desc;
  m->x = x;
  m->w = DevWeights{};
  blob_layout(x, static_cast<const float*>(d_mem), &m->w, kTensorAlign);
  m->w.prec = desc->prec == PSWA_BF16 ? PSWA_PREC_BF16
              : desc->prec == PSWA_FP8_E4M3 ? PSWA_PREC_FP8 : PSWA_PREC_F32;
  m->w.kv16 = desc->prec != PSWA_FP32;  // reduced-precision models keep K/V in BF16
  assign_slots(m->w, x);
  std::vector<std::vector<uint8_t>> staging;
  if (desc->prec != PSWA_FP32) {
    std::vector<std::pair<int, size_t>> qoff;
    device_layout(*desc, &qoff);
    auto targets = quant_targets(m->w, x);
    for (size_t i = 0; i < targets.size(); ++i) {
      const float* w = h_blob + src[targets[i].tensor].first;
      const size_t n = src[targets[i].tensor].second;
      const size_t K = targets[i].K, N = n / K;
      if (N * K != n || N % 8 != 0 || K % 32 != 0) {
        (void)hipStreamSynchronize(st);  // copies from host buffers still in flight
        return fail(PSWA_E_UNSUPPORTED, "projection %d of %zu values is not [8a][32b]",
                    targets[i].tensor, n);
      }
      std::vector<uint8_t> q;
      float inv = 1.f;
      if (desc->prec == PSWA_BF16) {
        q.resize(2 * n);
        for (size_t k = 0; k < n; ++k) {
          const uint16_t h = bf16_rne_host(w[k]);
          std::memcpy(&q[2 * k], &h, 2);
        }
      } else {
        double amax = 0;
        for (size_t k = 0; k < n; ++k) amax = std::max(amax, std::fabs(double(w[k])));
        const double sc = amax > 0 ? 448.0 / amax : 1.0;  // static per-tensor scale
        q.resize(n);
        for (size_t k = 0; k < n; ++k) q[k] = fp8_e4m3_rne_host(float(double(w[k]) * sc));
        inv = float(1.0 / sc);
      }
      q = to_fragment_layout(q, N, K, desc->prec == PSWA_BF16 ? 2 : 1);
      char* dst = static_cast<char*>(d_mem) + qoff[i].second;
      PSWA_HIP_TRY(hipMemcpyAsync(dst, q.data(), q.size(), hipMemcpyHostToDevice, st));
      QW& qw = *targets[i].dst;
      qw.q = dst;
      qw.inv_scale = inv;
      if (has_act_maxima(*desc)) {  // static per-tensor activation scale
        const double amax = h_blob[nweights + qw.slot];
        qw.ascale = amax > 0 ? float(448.0 / amax) : 1.0f;
      }
      staging.push_back(std::move(q));
    }
  }
  if (x.cg) {  // compacted per-group copies of the masked maps
    std::vector<size_t> wy_off, m_off;
    device_layout(*desc, nullptr, &wy_off, &m_off);
    const size_t base = 12 + 8 * (size_t)x.L;  // first Channel Transformer tensor
    const float* Wy = h_blob + src[base + 3].first;
    const size_t dg = x.cdg, Cg = x.cCg, C = x.C, dc = x.cd;
    // (each host copy lives in `staging` until the uploads are waited for)
    auto host_copy = [&](size_t floats) {
      staging.emplace_back(floats * sizeof(float));
      return reinterpret_cast<float*>(staging.back().data());
    };
    for (int g = 1; g < x.cg; ++g) {
      // rows of group g over latent groups 0 .. g-1: latent column c sits
      // at column c + Cg of the shifted input
      const size_t n = dg * g * Cg;
      float* q = host_copy(n);
      for (size_t r = 0; r < dg; ++r)
        for (size_t c = 0; c < g * Cg; ++c) q[r * g * Cg + c] = Wy[(g * dg + r) * C + c + Cg];
      char* dst = static_cast<char*>(d_mem) + wy_off[g];
      PSWA_HIP_TRY(hipMemcpyAsync(dst, q, n * sizeof(float), hipMemcpyHostToDevice, st));
      m->w.ct.wy_g[g] = reinterpret_cast<const float*>(dst);
    }
    for (int b = 0; b < x.cL; ++b) {
      const float* Mb = h_blob + src[base + 5 + 6 * b].first;
      for (int g = 0; g < x.cg; ++g) {
        const size_t k = (g + 1) * dg;
        float* q = host_copy(dg * k);
        for (size_t r = 0; r < dg; ++r)
          for (size_t c = 0; c < k; ++c) q[r * k + c] = Mb[(g * dg + r) * dc + c];
        char* dst = static_cast<char*>(d_mem) + m_off[b * x.cg + g];
        PSWA_HIP_TRY(hipMemcpyAsync(dst, q, dg * k * sizeof(float), hipMemcpyHostToDevice, st));
        m->w.ct.m_g[b][g] = reinterpret_cast<const float*>(dst);
      }
    }
  }
  PSWA_HIP_TRY(hipStreamSynchronize(st));
  *out = m.release();
  return PSWA_OK;
}

void pswa_model_destroy(pswa_model* model) { delete model; }

pswa_status pswa_quantize(int prec, const float* h_in, size_t n, void* h_out, float* h_inv_scale) {
  if ((n && (!h_in || !h_out)) || !h_inv_scale) return fail(PSWA_E_ARG, "null pointer argument");
  if (prec == PSWA_BF16) {
    uint16_t* o = static_cast<uint16_t*>(h_out);
    for (size_t k = 0; k < n; ++k) o[k] = bf16_rne_host(h_in[k]);
    *h_inv_scale = 1.f;
    return PSWA_OK;
  }
  if (prec == PSWA_FP8_E4M3) {
    double amax = 0;
    for (size_t k = 0; k < n; ++k) amax = std::max(amax, std::fabs(double(h_in[k])));
    const double sc = amax > 0 ? 448.0 / amax : 1.0;
    uint8_t* o = static_cast<uint8_t*>(h_out);
    for (size_t k = 0; k < n; ++k) o[k] = fp8_e4m3_rne_host(float(double(h_in[k]) * sc));
    *h_inv_scale = float(1.0 / sc);
    return PSWA_OK;
  }
  return fail(PSWA_E_ARG, "precision %d has no quantized form", prec);
}

size_t pswa_encode_workspace_bytes(const pswa_model* model, const pswa_frame_desc* frame) {
  std::string why;
  if (!model || !valid_frame(frame, &why)) return 0;
  return plan_encode(model->x, *frame, nullptr).bytes;
}

}  // extern "C"

namespace {

pswa_status encode_impl(const pswa_model* model, const pswa_frame_desc* frame,
                        const int32_t* d_latents, const int32_t* d_hyper,
                        const int32_t* d_prev, float* d_mean, float* d_scale,
                        float* d_bits, int32_t* d_cdf_center, uint16_t* d_cdf_index,
                        double* h_total_bits, void* d_ws, size_t ws_bytes, void* stream) {
  std::string why;
  if (!model) return fail(PSWA_E_ARG, "model is null");
  if (!valid_frame(frame, &why)) return fail(PSWA_E_SHAPE, "invalid frame: %s", why.c_str());
  if (!d_latents || !d_hyper || !d_mean || !d_scale || !d_bits || !d_cdf_center || !d_cdf_index || !d_ws)
    return fail(PSWA_E_ARG, "null pointer argument");
  if (frame->n_prev == 2 && !d_prev) return fail(PSWA_E_ARG, "P-frame needs d_prev");
  if (frame->n_prev == 0 && d_prev) return fail(PSWA_E_ARG, "I-frame must pass d_prev = NULL");
  if ((reinterpret_cast<uintptr_t>(d_ws) % kAlign) != 0)
    return fail(PSWA_E_ARG, "workspace must be 256-byte aligned");
  const NetDims& x = model->x;
  EncodeWs ws = plan_encode(x, *frame, d_ws);
  if (ws_bytes < ws.bytes) return fail(PSWA_E_ARG, "workspace %zu bytes < %zu", ws_bytes, ws.bytes);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int HW = frame->H * frame->W;

  zero_ints(ws.flag, 1, st);
  hyper_embed(d_hyper, frame->Hh, frame->Wh, x.Ch, model->w.hyperW, model->w.P4, frame->H,
              frame->W, x.d, ws.h, st);
  null_row(ws.acc_kv, HW, model->w.knull, model->w.vnull, x.d, model->w.kv16, st);
  PassCtx c = frame_ctx(*frame);
  c.M = HW;
  c.h = ws.h;
  c.acc_kv = ws.acc_kv;
  c.kv = ws.kv;
  c.kv_stride = 0;  // one K/V buffer, refilled layer by layer
  c.tkv = frame->n_prev ? ws.tkv : nullptr;
  c.tkv_stride = 0;
  c.x = ws.a.x; c.q = ws.a.q; c.att = ws.a.att; c.e = ws.a.e; c.t1 = ws.a.t1; c.hmid = ws.a.hmid;
  c.ct_c = ws.a.ct_c; c.ct_u = ws.a.ct_u; c.ct_h = ws.a.ct_h; c.ct_t1 = ws.a.ct_t1;
  c.mean = d_mean; c.scale = d_scale; c.bits = d_bits; c.center = d_cdf_center;
  c.index = d_cdf_index; c.flag = ws.flag;
  c.ydec = const_cast<int32_t*>(d_latents);  // only read: the encoder knows every symbol
  run_embed(model, c, st);
  if (frame->n_prev) embed_prev(model, HW, HW, 0, d_prev, ws.e_prev, st);
  const bool pf = frame->n_prev != 0;
  run_pass(
      model, c,
      [&](int l) {
        if (pf) temporal_kv_layer(model, HW, HW, 0, ws.e_prev, l, ws.tkv, st);
      },
      [](int) {}, st);
  symbol_bits(nullptr, HW, x.C, d_latents, d_mean, d_scale, d_bits, st);
  PSWA_HIP_TRY(hipGetLastError());
  if (h_total_bits)
    return finish_sum(d_bits, (size_t)HW * x.C, ws.sum, ws.flag, h_total_bits, st);
  return PSWA_OK;
}

// Per-symbol outputs a calibration run writes and discards, after the encode
// workspace.
struct CalibOut {
  float *mean, *scale, *bits;
  int32_t* center;
  uint16_t* index;
  size_t bytes;
};
CalibOut plan_calib(size_t n, void* base) {
  Layout L(base);
  CalibOut o;
  o.mean = L.take<float>(n);
  o.scale = L.take<float>(n);
  o.bits = L.take<float>(n);
  o.center = L.take<int32_t>(n);
  o.index = L.take<uint16_t>(n);
  o.bytes = L.used;
  return o;
}

}  // namespace

namespace pswa {
pswa_status encode_into(const pswa_model* model, const pswa_frame_desc* frame,
                        const int32_t* d_latents, const int32_t* d_hyper, const int32_t* d_prev,
                        float* d_mean, float* d_scale, float* d_bits, int32_t* d_cdf_center,
                        uint16_t* d_cdf_index, double* h_total_bits, void* d_ws, size_t ws_bytes,
                        void* stream) {
  return encode_impl(model, frame, d_latents, d_hyper, d_prev, d_mean, d_scale, d_bits,
                     d_cdf_center, d_cdf_index, h_total_bits, d_ws, ws_bytes, stream);
}
}  // namespace pswa

extern "C" {

pswa_status pswa_encode_params(const pswa_model* model, const pswa_frame_desc* frame,
                               const int32_t* d_latents, const int32_t* d_hyper,
                               const int32_t* d_prev, float* d_mean, float* d_scale,
                               float* d_bits, int32_t* d_cdf_center, uint16_t* d_cdf_index,
                               double* h_total_bits, void* d_ws, size_t ws_bytes, void* stream) {
  return encode_impl(model, frame, d_latents, d_hyper, d_prev, d_mean, d_scale, d_bits,
                     d_cdf_center, d_cdf_index, h_total_bits, d_ws, ws_bytes, stream);
}

size_t pswa_calibrate_workspace_bytes(const pswa_model* model, const pswa_frame_desc* frame) {
  std::string why;
  if (!model || !valid_frame(frame, &why)) return 0;
  const size_t n = (size_t)frame->H * frame->W * model->x.C;
  return align_up(plan_encode(model->x, *frame, nullptr).bytes) + plan_calib(n, nullptr).bytes;
}

pswa_status pswa_calibrate(const pswa_model* model, const pswa_frame_desc* frame,
                           const int32_t* d_latents, const int32_t* d_hyper,
                           const int32_t* d_prev, float* d_amax, void* d_ws, size_t ws_bytes,
                           void* stream) {
  std::string why;
  if (!model) return fail(PSWA_E_ARG, "model is null");
  if (model->desc.prec != PSWA_FP32)
    return fail(PSWA_E_UNSUPPORTED, "calibration runs on an FP32 model");
  if (!valid_frame(frame, &why)) return fail(PSWA_E_SHAPE, "invalid frame: %s", why.c_str());
  if (!d_amax || !d_ws) return fail(PSWA_E_ARG, "null pointer argument");
  if ((reinterpret_cast<uintptr_t>(d_ws) % kAlign) != 0)
    return fail(PSWA_E_ARG, "workspace must be 256-byte aligned");
  const size_t need = pswa_calibrate_workspace_bytes(model, frame);
  if (ws_bytes < need) return fail(PSWA_E_ARG, "workspace %zu bytes < %zu", ws_bytes, need);
  const size_t enc = align_up(plan_encode(model->x, *frame, nullptr).bytes);
  const size_t n = (size_t)frame->H * frame->W * model->x.C;
  CalibOut o = plan_calib(n, static_cast<char*>(d_ws) + enc);
  pswa_model rec = *model;  // the same weights, recording each input's maximum
  rec.w.calib = d_amax;
  return encode_impl(&rec, frame, d_latents, d_hyper, d_prev, o.mean, o.scale, o.bits, o.center,
                     o.index, nullptr, d_ws, enc, stream);
}

size_t pswa_state_bytes(const pswa_model* model, const pswa_frame_desc* frame) {
  std::string why;
  if (!model || !valid_frame(frame, &why)) return 0;
  pswa_state tmp;
  plan_state(model->x, *frame, nullptr, &tmp);
  return tmp.bytes;
}

pswa_status pswa_decode_begin(const pswa_model* model, const pswa_frame_desc* frame,
                              const int32_t* d_hyper, const int32_t* d_prev, int symbol_source,
                              const void* src, size_t src_bytes, void* d_state_mem,
                              size_t state_bytes, void* stream, pswa_state** out) {
  std::string why;
  if (!out) return fail(PSWA_E_ARG, "out is null");
  *out = nullptr;
  if (!model) return fail(PSWA_E_ARG, "model is null");
  if (!valid_frame(frame, &why)) return fail(PSWA_E_SHAPE, "invalid frame: %s", why.c_str());
  if (!d_hyper || !src || !d_state_mem) return fail(PSWA_E_ARG, "null pointer argument");
  if (symbol_source != PSWA_SRC_DEVICE && symbol_source != PSWA_SRC_BITSTREAM)
    return fail(PSWA_E_ARG, "unknown symbol source %d", symbol_source);
  if (symbol_source == PSWA_SRC_BITSTREAM && model->x.cg)
    return fail(PSWA_E_UNSUPPORTED,
                "bitstream decoding of models with channel groups is not built (device source only)");
  if (frame->n_prev == 2 && !d_prev) return fail(PSWA_E_ARG, "P-frame needs d_prev");
  if (frame->n_prev == 0 && d_prev) return fail(PSWA_E_ARG, "I-frame must pass d_prev = NULL");
  if ((reinterpret_cast<uintptr_t>(d_state_mem) % kAlign) != 0)
    return fail(PSWA_E_ARG, "state memory must be 256-byte aligned");
  std::unique_ptr<pswa_state> S(new pswa_state);
  plan_state(model->x, *frame, d_state_mem, S.get());
  if (state_bytes < S->bytes) return fail(PSWA_E_ARG, "state %zu bytes < %zu", state_bytes, S->bytes);
  S->model = model;
  S->f = *frame;
  S->source = symbol_source;
  const NetDims& x = model->x;
  S->start.assign(S->T + 1, 0);
  for (int t = 0; t < S->T; ++t)
    S->start[t + 1] = S->start[t] + sched_len(x, frame->H, frame->W, t);
  if (symbol_source == PSWA_SRC_DEVICE) {
    S->d_src = static_cast<const int32_t*>(src);
  } else {
    const uint8_t* b = static_cast<const uint8_t*>(src);
    S->stream.assign(b, b + src_bytes);
    S->dec.reset(new RangeDecoder(S->stream.data(), S->stream.size()));
    const size_t n = (size_t)S->nmax * x.C;
    PSWA_HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&S->h_cc), n * sizeof(int32_t), hipHostMallocDefault));
    PSWA_HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&S->h_ci), n * sizeof(uint16_t), hipHostMallocDefault));
    PSWA_HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&S->h_sym), n * sizeof(int32_t), hipHostMallocDefault));
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int HW = frame->H * frame->W;
  zero_ints(S->flag, 1, st);
  {  // positions in decode order (step by step)
    std::vector<int> pos;
    pos.reserve(HW);
    for (int t = 0; t < S->T; ++t)
      sched_for_each(x, frame->H, frame->W, t, [&](int i, int j) { pos.push_back(i * frame->W + j); });
    PSWA_HIP_TRY(hipMemcpyAsync(S->pos_all, pos.data(), pos.size() * sizeof(int),
                                hipMemcpyHostToDevice, st));
    PSWA_HIP_TRY(hipStreamSynchronize(st));
  }
  hyper_embed(d_hyper, frame->Hh, frame->Wh, x.Ch, model->w.hyperW, model->w.P4, frame->H,
              frame->W, x.d, S->h, st);
  null_row(S->acc_kv, HW, model->w.knull, model->w.vnull, x.d, model->w.kv16, st);
  if (frame->n_prev) {
    embed_prev(model, HW, HW, 0, d_prev, S->e_prev, st);
    for (int l = 0; l < x.L; ++l)
      temporal_kv_layer(model, HW, HW, 0, S->e_prev, l, S->tkv + (size_t)l * 2 * HW * 2 * x.d, st);
  }
  PSWA_HIP_TRY(hipGetLastError());
  *out = S.release();
  return PSWA_OK;
}

int pswa_num_steps(const pswa_state* state) { return state ? state->T : -1; }

pswa_status pswa_decode_step(pswa_state* S, int t, void* stream) {
  if (!S) return fail(PSWA_E_ARG, "state is null");
  if (t != S->next_t)
    return fail(PSWA_E_ORDER, "decode_step(%d) called, next step is %d", t, S->next_t);
  if (t >= S->T) return fail(PSWA_E_ORDER, "all %d steps already decoded", S->T);
  const pswa_model* m = S->model;
  const NetDims& x = m->x;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int HW = S->f.H * S->f.W;
  const int n = S->start[t + 1] - S->start[t];
  const int* pos = S->pos_all + S->start[t];
  const bool bs = S->source == PSWA_SRC_BITSTREAM;

  PassCtx c = frame_ctx(S->f);
  c.M = n;
  c.gpos = pos;
  c.h = S->h;
  c.acc_kv = S->acc_kv;
  c.kv = S->kv;
  c.kv_stride = (size_t)HW * 2 * x.d;
  c.tkv = S->tkv;
  c.tkv_stride = (size_t)2 * HW * 2 * x.d;
  c.x = S->a.x; c.q = S->a.q; c.att = S->a.att; c.e = S->a.e; c.t1 = S->a.t1; c.hmid = S->a.hmid;
  c.ct_c = S->a.ct_c; c.ct_u = S->a.ct_u; c.ct_h = S->a.ct_h; c.ct_t1 = S->a.ct_t1;
  c.mean = S->mean; c.scale = S->scale; c.bits = S->bits; c.center = S->center;
  c.index = S->index; c.flag = S->flag;
  c.center_c = bs ? S->cc : nullptr;
  c.index_c = bs ? S->ci : nullptr;
  c.ydec = S->ydec;
  if (x.cg) {
    // channel groups one after the other, each group's symbols read before
    // the next group is predicted (device symbol source)
    run_pass(m, c, [](int) {},
             [&](int g) { gather_symbols(S->d_src, 0, pos, n, x.C, S->ydec, st, g * x.cCg, x.cCg); },
             st);
  } else {
    run_pass(m, c, [](int) {}, [](int) {}, st);
  }

  if (x.cg) {
    // (symbols already gathered group by group)
  } else if (!bs) {
    gather_symbols(S->d_src, 0, pos, n, x.C, S->ydec, st);
  } else {
    const size_t cnt = (size_t)n * x.C;
    PSWA_HIP_TRY(hipMemcpyAsync(S->h_cc, S->cc, cnt * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    PSWA_HIP_TRY(hipMemcpyAsync(S->h_ci, S->ci, cnt * sizeof(uint16_t), hipMemcpyDeviceToHost, st));
    PSWA_HIP_TRY(hipStreamSynchronize(st));
    for (size_t k = 0; k < cnt; ++k) {
      if (!S->dec->symbol(S->h_cc[k], S->h_ci[k], &S->h_sym[k]))
        return fail(PSWA_E_CORRUPT, "bitstream corrupt or truncated at step %d", t);
    }
    PSWA_HIP_TRY(hipMemcpyAsync(S->csym, S->h_sym, cnt * sizeof(int32_t), hipMemcpyHostToDevice, st));
    gather_symbols(S->csym, 1, pos, n, x.C, S->ydec, st);
  }
  symbol_bits(pos, n, x.C, S->ydec, S->mean, S->scale, S->bits, st);
  run_embed(m, c, st);
  PSWA_HIP_TRY(hipGetLastError());
  S->next_t = t + 1;
  return PSWA_OK;
}

pswa_status pswa_decode_end(pswa_state* S, int32_t* d_latents_out, float* d_mean, float* d_scale,
                            float* d_bits, int32_t* d_cdf_center, uint16_t* d_cdf_index,
                            double* h_total_bits, void* stream) {
  if (!S) return fail(PSWA_E_ARG, "state is null");
  if (S->next_t != S->T)
    return fail(PSWA_E_ORDER, "decode_end after %d of %d steps", S->next_t, S->T);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t n = (size_t)S->f.H * S->f.W * S->model->x.C;
  auto cp = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    return dst ? hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st) : hipSuccess;
  };
  PSWA_HIP_TRY(cp(d_latents_out, S->ydec, n * sizeof(int32_t)));
  PSWA_HIP_TRY(cp(d_mean, S->mean, n * sizeof(float)));
  PSWA_HIP_TRY(cp(d_scale, S->scale, n * sizeof(float)));
  PSWA_HIP_TRY(cp(d_bits, S->bits, n * sizeof(float)));
  PSWA_HIP_TRY(cp(d_cdf_center, S->center, n * sizeof(int32_t)));
  PSWA_HIP_TRY(cp(d_cdf_index, S->index, n * sizeof(uint16_t)));
  if (h_total_bits) return finish_sum(S->bits, n, S->sum, S->flag, h_total_bits, st);
  return PSWA_OK;
}

void pswa_state_destroy(pswa_state* state) { delete state; }

pswa_status pswa_cdf_select(const float* d_mean, const float* d_log_scale, size_t n,
                            int32_t* d_center, uint16_t* d_index, void* stream) {
  if (n == 0) return PSWA_OK;
  if (!d_mean || !d_log_scale || !d_center || !d_index) return fail(PSWA_E_ARG, "null pointer argument");
  cdf_select(d_mean, d_log_scale, n, ln_sigma_min_f32(), inv_delta_f32(), d_center, d_index,
             static_cast<hipStream_t>(stream));
  PSWA_HIP_TRY(hipGetLastError());
  return PSWA_OK;
}

pswa_status pswa_cdf_tables(uint32_t* h_radius, uint32_t* h_offset, uint16_t* h_freq,
                            size_t freq_cap) {
  if (!h_offset) return fail(PSWA_E_ARG, "h_offset is null");
  const CdfTables& t = cdf_tables();
  std::copy(t.offset.begin(), t.offset.end(), h_offset);
  if (h_radius) std::copy(t.radius.begin(), t.radius.end(), h_radius);
  if (h_freq) {
    if (freq_cap < t.freq.size())
      return fail(PSWA_E_ARG, "freq capacity %zu < %zu", freq_cap, t.freq.size());
    std::copy(t.freq.begin(), t.freq.end(), h_freq);
  }
  return PSWA_OK;
}

pswa_status pswa_range_encode_seq(size_t n, const int32_t* h_symbols, const int32_t* h_center,
                                  const uint16_t* h_index, uint8_t* out, size_t cap,
                                  size_t* out_bytes) {
  if (!out_bytes || (n && (!h_symbols || !h_center || !h_index)) || (cap && !out))
    return fail(PSWA_E_ARG, "null pointer argument");
  for (size_t k = 0; k < n; ++k)
    if (h_index[k] >= kTables) return fail(PSWA_E_ARG, "table index %u out of range", h_index[k]);
  RangeEncoder enc(out, cap);
  for (size_t k = 0; k < n; ++k) enc.symbol(h_symbols[k], h_center[k], h_index[k]);
  enc.finish();
  *out_bytes = enc.bytes();
  if (enc.overflow()) return fail(PSWA_E_ARG, "output capacity %zu < %zu bytes", cap, enc.bytes());
  return PSWA_OK;
}

pswa_status pswa_range_decode_seq(const uint8_t* in, size_t in_bytes, size_t n,
                                  const int32_t* h_center, const uint16_t* h_index,
                                  int32_t* h_symbols_out) {
  if ((n && (!h_center || !h_index || !h_symbols_out)) || (in_bytes && !in))
    return fail(PSWA_E_ARG, "null pointer argument");
  RangeDecoder dec(in, in_bytes);
  for (size_t k = 0; k < n; ++k)
    if (!dec.symbol(h_center[k], h_index[k], &h_symbols_out[k]))
      return fail(PSWA_E_CORRUPT, "bitstream corrupt or truncated at symbol %zu", k);
  return PSWA_OK;
}

pswa_status pswa_range_encode(const pswa_frame_desc* frame, int32_t C, int32_t window,
                              int32_t cycle, const int32_t* h_symbols, const int32_t* h_center,
                              const uint16_t* h_index, uint8_t* out, size_t cap,
                              size_t* out_bytes) {
  if (!frame || !h_symbols || !h_center || !h_index || !out_bytes || (cap && !out))
    return fail(PSWA_E_ARG, "null pointer argument");
  if (C < 1 || window < 3 || window % 2 == 0 || frame->H < 1 || frame->W < 1)
    return fail(PSWA_E_SHAPE, "invalid C, window or frame size");
  if (cycle != 0 && (cycle < 2 || cycle > 16))
    return fail(PSWA_E_ARG, "cycle must be 0 or in [2, 16]");
  NetDims x{};
  x.r = (window - 1) / 2;
  x.cycle = cycle;
  x.s = cycle ? cycle : x.r + 1;
  const int H = frame->H, W = frame->W;
  RangeEncoder enc(out, cap);
  const int T = sched_steps(x, H, W);
  bool bad = false;
  uint16_t bad_index = 0;
  for (int t = 0; t < T && !bad; ++t)
    sched_for_each(x, H, W, t, [&](int i, int j) {
      const size_t base = ((size_t)i * W + j) * C;
      for (int c = 0; c < C && !bad; ++c) {
        if (h_index[base + c] >= kTables) {
          bad = true;
          bad_index = h_index[base + c];
          return;
        }
        enc.symbol(h_symbols[base + c], h_center[base + c], h_index[base + c]);
      }
    });
  if (bad) return fail(PSWA_E_ARG, "table index %u out of range", bad_index);
  enc.finish();
  *out_bytes = enc.bytes();
  if (enc.overflow()) return fail(PSWA_E_ARG, "output capacity %zu < %zu bytes", cap, enc.bytes());
  return PSWA_OK;
}

}  // extern "C"
