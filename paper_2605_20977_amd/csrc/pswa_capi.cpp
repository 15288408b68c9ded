// C ABI and host runtime of the wavefront context model (see include/pswa.h).
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
#include "pswa_internal.h"

using namespace pswa;

namespace {

thread_local std::string g_last_error;

pswa_status fail(pswa_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(PSWA_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));      \
  } while (0)

constexpr size_t kAlign = 256;
constexpr size_t kTensorAlign = 64;  // floats
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

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

bool valid_desc(const pswa_model_desc* d, std::string* why) {
  if (!d) return *why = "null model desc", false;
  if (d->L < 1 || d->L > 64) return *why = "L out of range [1, 64]", false;
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
  return true;
}

struct Dims {
  int L, d, heads, dh, r, k, s, F, C, Ch, n_acc, n_sp, n_tm;
};

Dims dims_of(const pswa_model_desc& m) {
  Dims x;
  x.L = m.L;
  x.d = m.d;
  x.heads = m.heads;
  x.dh = m.d / m.heads;
  x.k = m.window;
  x.r = (m.window - 1) / 2;
  x.s = x.r + 1;
  x.F = m.mlp_ratio * m.d;
  x.C = m.C;
  x.Ch = m.Ch;
  x.n_acc = 2 * x.r * (x.r + 1);
  x.n_sp = x.n_acc + 1;
  x.n_tm = 2 * (2 * x.r + 1) * (2 * x.r + 1);
  return x;
}

struct LayerW {
  const float *g1, *Wqkv, *bias, *Wo, *g2, *Wgate, *Wup, *Wdown;
};

struct Weights {
  const float *hyperW, *P4, *ing, *inW, *acc_gq, *acc_Wq, *acc_gkv, *acc_Wkv, *knull, *vnull,
      *acc_bias, *acc_Wo;
  std::vector<LayerW> layers;
  const float *head_g, *W1, *W2, *gmu, *bmu, *gsig, *bsig;
};

// Walks the documented blob order; with base == nullptr it only counts.
// align > 1 pads every tensor to a multiple of `align` floats (the device
// layout keeps each tensor 256-byte aligned for vector loads).
size_t blob_layout(const Dims& x, const float* base, Weights* w, size_t align = 1,
                   std::vector<std::pair<size_t, size_t>>* spans = nullptr) {
  size_t off = 0;
  auto t = [&](size_t n) {
    const float* p = base ? base + off : nullptr;
    if (spans) spans->emplace_back(off, n);
    off += (n + align - 1) / align * align;
    return p;
  };
  const size_t d = x.d, C = x.C, Ch = x.Ch, F = x.F, h = x.heads;
  Weights tmp;
  Weights& W = w ? *w : tmp;
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
  W.layers.assign(x.L, LayerW{});
  for (int l = 0; l < x.L; ++l) {
    LayerW& L = W.layers[l];
    L.g1 = t(d);
    L.Wqkv = t(3 * d * d);
    L.bias = t(h * (x.n_sp + x.n_tm));
    L.Wo = t(d * d);
    L.g2 = t(d);
    L.Wgate = t(F * d);
    L.Wup = t(F * d);
    L.Wdown = t(d * F);
  }
  W.head_g = t(d);
  W.W1 = t(d * d);
  W.W2 = t(2 * C * d);
  W.gmu = t(C);
  W.bmu = t(C);
  W.gsig = t(C);
  W.bsig = t(C);
  return off;
}

}  // namespace

struct pswa_model {
  pswa_model_desc desc;
  Dims x;
  Weights w;
  float ln_smin, ln_smax, inv_delta;
};

namespace {

bool valid_frame(const pswa_model* m, const pswa_frame_desc* f, std::string* why) {
  if (!f) return *why = "null frame desc", false;
  if (f->H < 1 || f->W < 1 || (int64_t)f->H * f->W > (1 << 24))
    return *why = "H, W must be >= 1 with H*W <= 2^24", false;
  if (f->Hh != (f->H + 3) / 4 || f->Wh != (f->W + 3) / 4)
    return *why = "hyperprior grid must be ceil(H/4) x ceil(W/4)", false;
  if (f->n_prev != 0 && f->n_prev != 2) return *why = "n_prev must be 0 or 2", false;
  (void)m;
  return true;
}

// Activation buffers for `rows` rows.
struct Acts {
  float *x, *q, *att, *e, *t1, *hmid;
};

Acts take_acts(Layout& L, const Dims& x, size_t rows) {
  Acts a;
  a.x = L.take<float>(rows * x.d);
  a.q = L.take<float>(rows * x.d);
  a.att = L.take<float>(rows * x.d);
  a.e = L.take<float>(rows * x.d);
  a.t1 = L.take<float>(rows * x.d);
  a.hmid = L.take<float>(rows * x.F);
  return a;
}

// Per-symbol outputs [HW][C].
struct SymOut {
  float *mean, *scale, *bits;
  int32_t* center;
  uint16_t* index;
};

// Everything one pass over a set of rows needs.
struct RowPass {
  int M;
  const int* pos;        // row -> position (null: identity)
  const float* h;        // hyper tokens [HW][d]
  float* acc_kv;         // [HW][2d]
  Acts a;
  SymOut out;
  int32_t* center_c;     // compact copies for the bitstream decoder (or null)
  uint16_t* index_c;
  int* flag;
};

struct FrameGeom {
  int H, W;
};

// Accumulator, L layers and head for the pass's rows. kv_of(l) gives layer
// l's K/V cache [HW][2d]; tkv_of(l) its temporal K/V [2][HW][2d] or null.
template <class KvOf, class TkvOf, class BeforeLayer>
void run_rows(const pswa_model* m, const FrameGeom& g, const RowPass& P, KvOf kv_of,
              TkvOf tkv_of, BeforeLayer before_layer, hipStream_t st) {
  const Dims& x = m->x;
  const Weights& w = m->w;
  const int d = x.d;

  // Accumulator: q from the hyper token, keys strictly past + null slot.
  GemmArgs q{};
  q.M = P.M; q.N = d; q.K = d;
  q.X = P.h; q.ldx = d; q.xrow = P.pos; q.gain = w.acc_gq; q.W = w.acc_Wq;
  q.Y = P.a.q; q.ldy = d;
  gemm_f32(A_FLOAT, true, EPI_STORE, q, st);

  AttnArgs at{};
  at.M = P.M; at.pos = P.pos; at.H = g.H; at.W = g.W; at.r = x.r; at.heads = x.heads;
  at.dh = x.dh; at.d = d; at.q = P.a.q; at.ldq = d; at.kv = P.acc_kv; at.tkv = nullptr;
  at.bias = w.acc_bias; at.nbias = x.n_acc; at.knull = w.knull; at.vnull = w.vnull;
  at.include_self = 0; at.out = P.a.att; at.ldo = d;
  attention_f32(at, st);

  GemmArgs o{};
  o.M = P.M; o.N = d; o.K = d;
  o.X = P.a.att; o.ldx = d; o.W = w.acc_Wo;
  o.R = P.h; o.ldr = d; o.rrow = P.pos; o.Y = P.a.x; o.ldy = d;
  gemm_f32(A_FLOAT, false, EPI_RESID, o, st);

  for (int l = 0; l < x.L; ++l) {
    const LayerW& L = w.layers[l];
    before_layer(l);
    float* kv = kv_of(l);
    GemmArgs a{};
    a.M = P.M; a.N = 3 * d; a.K = d;
    a.X = P.a.x; a.ldx = d; a.gain = L.g1; a.W = L.Wqkv;
    a.Y = P.a.q; a.ldy = d; a.Y2 = kv; a.ldy2 = 2 * d; a.y2row = P.pos; a.nsplit = d;
    gemm_f32(A_FLOAT, true, EPI_QKV, a, st);

    AttnArgs la = at;
    la.kv = kv; la.tkv = tkv_of(l); la.bias = L.bias; la.nbias = x.n_sp + x.n_tm;
    la.knull = nullptr; la.vnull = nullptr; la.include_self = 1;
    attention_f32(la, st);

    GemmArgs b{};
    b.M = P.M; b.N = d; b.K = d;
    b.X = P.a.att; b.ldx = d; b.W = L.Wo; b.R = P.a.x; b.ldr = d; b.Y = P.a.x; b.ldy = d;
    gemm_f32(A_FLOAT, false, EPI_RESID, b, st);

    GemmArgs c{};
    c.M = P.M; c.N = x.F; c.K = d;
    c.X = P.a.x; c.ldx = d; c.gain = L.g2; c.W = L.Wgate; c.W2 = L.Wup;
    c.Y = P.a.hmid; c.ldy = x.F;
    gemm_f32(A_FLOAT, true, EPI_SWIGLU, c, st);

    GemmArgs e{};
    e.M = P.M; e.N = d; e.K = x.F;
    e.X = P.a.hmid; e.ldx = x.F; e.W = L.Wdown; e.R = P.a.x; e.ldr = d; e.Y = P.a.x; e.ldy = d;
    gemm_f32(A_FLOAT, false, EPI_RESID, e, st);
  }

  GemmArgs h1{};
  h1.M = P.M; h1.N = d; h1.K = d;
  h1.X = P.a.x; h1.ldx = d; h1.gain = w.head_g; h1.W = w.W1; h1.Y = P.a.t1; h1.ldy = d;
  gemm_f32(A_FLOAT, true, EPI_SILU, h1, st);

  GemmArgs h2{};
  h2.M = P.M; h2.N = x.C; h2.K = d;
  h2.X = P.a.t1; h2.ldx = d; h2.W = w.W2; h2.W2 = w.W2 + (size_t)x.C * d; h2.yrow = P.pos;
  h2.head.gmu = w.gmu; h2.head.bmu = w.bmu; h2.head.gsig = w.gsig; h2.head.bsig = w.bsig;
  h2.head.ln_smin = m->ln_smin; h2.head.ln_smax = m->ln_smax; h2.head.inv_delta = m->inv_delta;
  h2.head.mean = P.out.mean; h2.head.scale = P.out.scale; h2.head.center = P.out.center;
  h2.head.index = P.out.index; h2.head.center_c = P.center_c; h2.head.index_c = P.index_c;
  h2.head.flag = P.flag;
  gemm_f32(A_FLOAT, false, EPI_HEAD, h2, st);
}

// Embedding of decoded latents (rows given by pos) and their accumulator K/V.
void embed_rows(const pswa_model* m, int M, const int* pos, const int32_t* lat, float* e,
                float* acc_kv, hipStream_t st) {
  const Dims& x = m->x;
  GemmArgs a{};
  a.M = M; a.N = x.d; a.K = x.C;
  a.Xi = lat; a.ldx = x.C; a.xrow = pos; a.xscale = m->w.ing; a.W = m->w.inW;
  a.Y = e; a.ldy = x.d;
  gemm_f32(A_INT, false, EPI_STORE, a, st);
  GemmArgs b{};
  b.M = M; b.N = 2 * x.d; b.K = x.d;
  b.X = e; b.ldx = x.d; b.gain = m->w.acc_gkv; b.W = m->w.acc_Wkv;
  b.Y = acc_kv; b.ldy = 2 * x.d; b.yrow = pos;
  gemm_f32(A_FLOAT, true, EPI_STORE, b, st);
}

// Layer-l temporal K/V of the two previous frames from their embeddings.
void temporal_kv_layer(const pswa_model* m, int HW, const float* e_prev, int l, float* tkv,
                       hipStream_t st) {
  const Dims& x = m->x;
  for (int tau = 0; tau < 2; ++tau) {
    GemmArgs a{};
    a.M = HW; a.N = 2 * x.d; a.K = x.d;
    a.X = e_prev + (size_t)tau * HW * x.d; a.ldx = x.d; a.gain = m->w.layers[l].g1;
    a.W = m->w.layers[l].Wqkv + (size_t)x.d * x.d;
    a.Y = tkv + (size_t)tau * HW * 2 * x.d; a.ldy = 2 * x.d;
    gemm_f32(A_FLOAT, true, EPI_STORE, a, st);
  }
}

void embed_prev(const pswa_model* m, int HW, const int32_t* prev, float* e_prev, hipStream_t st) {
  const Dims& x = m->x;
  for (int tau = 0; tau < 2; ++tau) {
    GemmArgs a{};
    a.M = HW; a.N = x.d; a.K = x.C;
    a.Xi = prev + (size_t)tau * HW * x.C; a.ldx = x.C; a.xscale = m->w.ing; a.W = m->w.inW;
    a.Y = e_prev + (size_t)tau * HW * x.d; a.ldy = x.d;
    gemm_f32(A_INT, false, EPI_STORE, a, st);
  }
}

// ------------------------------------------------------------ encode ws
struct EncodeWs {
  float* h;
  float* acc_kv;
  float* kv;
  float* tkv;
  float* e_prev;
  Acts a;
  int* flag;
  float* sum;
  size_t bytes;
};

EncodeWs plan_encode(const Dims& x, const pswa_frame_desc& f, void* base) {
  Layout L(base);
  const size_t HW = (size_t)f.H * f.W;
  EncodeWs w;
  w.h = L.take<float>(HW * x.d);
  w.acc_kv = L.take<float>(HW * 2 * x.d);
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
  SymOut out;
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

int steps_of(int H, int W, int s) { return (W - 1) + s * (H - 1) + 1; }

int diag_len(int H, int W, int s, int t) {
  int n = 0;
  for (int i = 0; i < H; ++i) {
    const int j = t - s * i;
    if (j >= 0 && j < W) ++n;
  }
  return n;
}

void plan_state(const Dims& x, const pswa_frame_desc& f, void* base, pswa_state* st) {
  Layout L(base);
  const size_t HW = (size_t)f.H * f.W;
  int nmax = 0;
  const int T = steps_of(f.H, f.W, x.s);
  // n_t is maximal on the diagonals where every row fits: min(H, ceil(W/s)) bounds it.
  nmax = std::min(f.H, (f.W + x.s - 1) / x.s);
  st->T = T;
  st->nmax = nmax;
  st->h = L.take<float>(HW * x.d);
  st->acc_kv = L.take<float>(HW * 2 * x.d);
  st->kv = L.take<float>((size_t)x.L * HW * 2 * x.d);
  st->tkv = f.n_prev ? L.take<float>((size_t)x.L * 2 * HW * 2 * x.d) : nullptr;
  st->e_prev = f.n_prev ? L.take<float>(2 * HW * x.d) : nullptr;
  st->ydec = L.take<int32_t>(HW * x.C);
  st->out.mean = L.take<float>(HW * x.C);
  st->out.scale = L.take<float>(HW * x.C);
  st->out.bits = L.take<float>(HW * x.C);
  st->out.center = L.take<int32_t>(HW * x.C);
  st->out.index = L.take<uint16_t>(HW * x.C);
  st->pos_all = L.take<int>(HW);
  st->a = take_acts(L, x, nmax);
  st->cc = L.take<int32_t>((size_t)nmax * x.C);
  st->ci = L.take<uint16_t>((size_t)nmax * x.C);
  st->csym = L.take<int32_t>((size_t)nmax * x.C);
  st->flag = L.take<int>(64);
  st->sum = L.take<float>(64);
  st->bytes = L.used;
}

pswa_status finish_sum(const float* bits, size_t n, float* d_sum, const int* d_flag,
                       double* h_total, hipStream_t st) {
  sum_f32(bits, n, d_sum, st);
  HIP_TRY(hipGetLastError());
  float s = 0.f;
  int flag = 0;
  HIP_TRY(hipMemcpyAsync(&s, d_sum, sizeof s, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(&flag, d_flag, sizeof flag, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  *h_total = double(s);
  if (flag) return fail(PSWA_E_NUMERIC, "non-finite mean or scale produced");
  return PSWA_OK;
}

}  // namespace

extern "C" {

const char* pswa_last_error(void) { return g_last_error.c_str(); }

size_t pswa_model_blob_floats(const pswa_model_desc* desc) {
  std::string why;
  if (!valid_desc(desc, &why)) return 0;
  return blob_layout(dims_of(*desc), nullptr, nullptr);
}

size_t pswa_model_device_bytes(const pswa_model_desc* desc) {
  std::string why;
  if (!valid_desc(desc, &why)) return 0;
  return align_up(blob_layout(dims_of(*desc), nullptr, nullptr, kTensorAlign) * sizeof(float));
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
  const Dims x = dims_of(*desc);
  const size_t need = blob_layout(x, nullptr, nullptr);
  if (blob_floats != need)
    return fail(PSWA_E_SHAPE, "blob has %zu floats, model needs %zu", blob_floats, need);
  if (d_bytes < pswa_model_device_bytes(desc))
    return fail(PSWA_E_ARG, "device region %zu bytes < %zu", d_bytes, pswa_model_device_bytes(desc));
  if (desc->prec != PSWA_FP32)
    return fail(PSWA_E_UNSUPPORTED, "precision %d is not built in this library", desc->prec);
  hipStream_t st = static_cast<hipStream_t>(stream);
  // Re-lay the blob with every tensor 256-byte aligned, then one upload.
  std::vector<std::pair<size_t, size_t>> src, dst;
  blob_layout(x, nullptr, nullptr, 1, &src);
  const size_t dev_floats = blob_layout(x, nullptr, nullptr, kTensorAlign, &dst);
  std::vector<float> padded(dev_floats, 0.f);
  for (size_t i = 0; i < src.size(); ++i)
    std::memcpy(padded.data() + dst[i].first, h_blob + src[i].first, src[i].second * sizeof(float));
  HIP_TRY(hipMemcpyAsync(d_mem, padded.data(), dev_floats * sizeof(float), hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  auto* m = new pswa_model;
  m->desc = *desc;
  m->x = x;
  blob_layout(x, static_cast<const float*>(d_mem), &m->w, kTensorAlign);
  m->ln_smin = ln_sigma_min_f32();
  m->ln_smax = float(std::log(kSigmaMax));
  m->inv_delta = inv_delta_f32();
  *out = m;
  return PSWA_OK;
}

void pswa_model_destroy(pswa_model* model) { delete model; }

size_t pswa_encode_workspace_bytes(const pswa_model* model, const pswa_frame_desc* frame) {
  std::string why;
  if (!model || !valid_frame(model, frame, &why)) return 0;
  return plan_encode(model->x, *frame, nullptr).bytes;
}

pswa_status pswa_encode_params(const pswa_model* model, const pswa_frame_desc* frame,
                               const int32_t* d_latents, const int32_t* d_hyper,
                               const int32_t* d_prev, float* d_mean, float* d_scale,
                               float* d_bits, int32_t* d_cdf_center, uint16_t* d_cdf_index,
                               double* h_total_bits, void* d_ws, size_t ws_bytes, void* stream) {
  std::string why;
  if (!model) return fail(PSWA_E_ARG, "model is null");
  if (!valid_frame(model, frame, &why)) return fail(PSWA_E_SHAPE, "invalid frame: %s", why.c_str());
  if (!d_latents || !d_hyper || !d_mean || !d_scale || !d_bits || !d_cdf_center || !d_cdf_index || !d_ws)
    return fail(PSWA_E_ARG, "null pointer argument");
  if (frame->n_prev == 2 && !d_prev) return fail(PSWA_E_ARG, "P-frame needs d_prev");
  if (frame->n_prev == 0 && d_prev) return fail(PSWA_E_ARG, "I-frame must pass d_prev = NULL");
  if ((reinterpret_cast<uintptr_t>(d_ws) % kAlign) != 0)
    return fail(PSWA_E_ARG, "workspace must be 256-byte aligned");
  const Dims& x = model->x;
  EncodeWs ws = plan_encode(x, *frame, d_ws);
  if (ws_bytes < ws.bytes) return fail(PSWA_E_ARG, "workspace %zu bytes < %zu", ws_bytes, ws.bytes);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int HW = frame->H * frame->W;
  const FrameGeom g{frame->H, frame->W};

  HIP_TRY(hipMemsetAsync(ws.flag, 0, sizeof(int), st));
  hyper_embed(d_hyper, frame->Hh, frame->Wh, x.Ch, model->w.hyperW, model->w.P4, frame->H,
              frame->W, x.d, ws.h, st);
  embed_rows(model, HW, nullptr, d_latents, ws.a.e, ws.acc_kv, st);
  if (frame->n_prev) embed_prev(model, HW, d_prev, ws.e_prev, st);

  RowPass P{};
  P.M = HW; P.pos = nullptr; P.h = ws.h; P.acc_kv = ws.acc_kv; P.a = ws.a;
  P.out = SymOut{d_mean, d_scale, d_bits, d_cdf_center, d_cdf_index};
  P.center_c = nullptr; P.index_c = nullptr; P.flag = ws.flag;
  const bool pf = frame->n_prev != 0;
  run_rows(
      model, g, P, [&](int) { return ws.kv; },
      [&](int) -> const float* { return pf ? ws.tkv : nullptr; },
      [&](int l) {
        if (pf) temporal_kv_layer(model, HW, ws.e_prev, l, ws.tkv, st);
      },
      st);
  symbol_bits(nullptr, HW, x.C, d_latents, d_mean, d_scale, d_bits, st);
  HIP_TRY(hipGetLastError());
  if (h_total_bits)
    return finish_sum(d_bits, (size_t)HW * x.C, ws.sum, ws.flag, h_total_bits, st);
  return PSWA_OK;
}

size_t pswa_state_bytes(const pswa_model* model, const pswa_frame_desc* frame) {
  std::string why;
  if (!model || !valid_frame(model, frame, &why)) return 0;
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
  if (!valid_frame(model, frame, &why)) return fail(PSWA_E_SHAPE, "invalid frame: %s", why.c_str());
  if (!d_hyper || !src || !d_state_mem) return fail(PSWA_E_ARG, "null pointer argument");
  if (symbol_source != PSWA_SRC_DEVICE && symbol_source != PSWA_SRC_BITSTREAM)
    return fail(PSWA_E_ARG, "unknown symbol source %d", symbol_source);
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
  const Dims& x = model->x;
  S->start.assign(S->T + 1, 0);
  for (int t = 0; t < S->T; ++t)
    S->start[t + 1] = S->start[t] + diag_len(frame->H, frame->W, x.s, t);
  if (symbol_source == PSWA_SRC_DEVICE) {
    S->d_src = static_cast<const int32_t*>(src);
  } else {
    const uint8_t* b = static_cast<const uint8_t*>(src);
    S->stream.assign(b, b + src_bytes);
    S->dec.reset(new RangeDecoder(S->stream.data(), S->stream.size()));
    const size_t n = (size_t)S->nmax * x.C;
    HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&S->h_cc), n * sizeof(int32_t), hipHostMallocDefault));
    HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&S->h_ci), n * sizeof(uint16_t), hipHostMallocDefault));
    HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&S->h_sym), n * sizeof(int32_t), hipHostMallocDefault));
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int HW = frame->H * frame->W;
  HIP_TRY(hipMemsetAsync(S->flag, 0, sizeof(int), st));
  fill_positions(frame->H, frame->W, x.s, S->pos_all, st);
  hyper_embed(d_hyper, frame->Hh, frame->Wh, x.Ch, model->w.hyperW, model->w.P4, frame->H,
              frame->W, x.d, S->h, st);
  if (frame->n_prev) {
    embed_prev(model, HW, d_prev, S->e_prev, st);
    for (int l = 0; l < x.L; ++l)
      temporal_kv_layer(model, HW, S->e_prev, l, S->tkv + (size_t)l * 2 * HW * 2 * x.d, st);
  }
  HIP_TRY(hipGetLastError());
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
  const Dims& x = m->x;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int HW = S->f.H * S->f.W;
  const int n = S->start[t + 1] - S->start[t];
  const int* pos = S->pos_all + S->start[t];
  const bool bs = S->source == PSWA_SRC_BITSTREAM;

  RowPass P{};
  P.M = n; P.pos = pos; P.h = S->h; P.acc_kv = S->acc_kv; P.a = S->a; P.out = S->out;
  P.center_c = bs ? S->cc : nullptr; P.index_c = bs ? S->ci : nullptr; P.flag = S->flag;
  run_rows(
      m, FrameGeom{S->f.H, S->f.W}, P,
      [&](int l) { return S->kv + (size_t)l * HW * 2 * x.d; },
      [&](int l) -> const float* {
        return S->tkv ? S->tkv + (size_t)l * 2 * HW * 2 * x.d : nullptr;
      },
      [](int) {}, st);

  if (!bs) {
    gather_symbols(S->d_src, 0, pos, n, x.C, S->ydec, st);
  } else {
    const size_t cnt = (size_t)n * x.C;
    HIP_TRY(hipMemcpyAsync(S->h_cc, S->cc, cnt * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(S->h_ci, S->ci, cnt * sizeof(uint16_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (size_t k = 0; k < cnt; ++k) {
      if (!S->dec->symbol(S->h_cc[k], S->h_ci[k], &S->h_sym[k]))
        return fail(PSWA_E_CORRUPT, "bitstream corrupt or truncated at step %d", t);
    }
    HIP_TRY(hipMemcpyAsync(S->csym, S->h_sym, cnt * sizeof(int32_t), hipMemcpyHostToDevice, st));
    gather_symbols(S->csym, 1, pos, n, x.C, S->ydec, st);
  }
  symbol_bits(pos, n, x.C, S->ydec, S->out.mean, S->out.scale, S->out.bits, st);
  embed_rows(m, n, pos, S->ydec, S->a.e, S->acc_kv, st);
  HIP_TRY(hipGetLastError());
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
  HIP_TRY(cp(d_latents_out, S->ydec, n * sizeof(int32_t)));
  HIP_TRY(cp(d_mean, S->out.mean, n * sizeof(float)));
  HIP_TRY(cp(d_scale, S->out.scale, n * sizeof(float)));
  HIP_TRY(cp(d_bits, S->out.bits, n * sizeof(float)));
  HIP_TRY(cp(d_cdf_center, S->out.center, n * sizeof(int32_t)));
  HIP_TRY(cp(d_cdf_index, S->out.index, n * sizeof(uint16_t)));
  if (h_total_bits) return finish_sum(S->out.bits, n, S->sum, S->flag, h_total_bits, st);
  return PSWA_OK;
}

void pswa_state_destroy(pswa_state* state) { delete state; }

pswa_status pswa_cdf_select(const float* d_mean, const float* d_log_scale, size_t n,
                            int32_t* d_center, uint16_t* d_index, void* stream) {
  if (n == 0) return PSWA_OK;
  if (!d_mean || !d_log_scale || !d_center || !d_index) return fail(PSWA_E_ARG, "null pointer argument");
  cdf_select(d_mean, d_log_scale, n, ln_sigma_min_f32(), inv_delta_f32(), d_center, d_index,
             static_cast<hipStream_t>(stream));
  HIP_TRY(hipGetLastError());
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
                              const int32_t* h_symbols, const int32_t* h_center,
                              const uint16_t* h_index, uint8_t* out, size_t cap,
                              size_t* out_bytes) {
  if (!frame || !h_symbols || !h_center || !h_index || !out_bytes || (cap && !out))
    return fail(PSWA_E_ARG, "null pointer argument");
  if (C < 1 || window < 3 || window % 2 == 0 || frame->H < 1 || frame->W < 1)
    return fail(PSWA_E_SHAPE, "invalid C, window or frame size");
  const int s = (window - 1) / 2 + 1;
  const int H = frame->H, W = frame->W;
  RangeEncoder enc(out, cap);
  const int T = steps_of(H, W, s);
  for (int t = 0; t < T; ++t)
    for (int i = 0; i < H; ++i) {
      const int j = t - s * i;
      if (j < 0 || j >= W) continue;
      const size_t base = ((size_t)i * W + j) * C;
      for (int c = 0; c < C; ++c) {
        if (h_index[base + c] >= kTables)
          return fail(PSWA_E_ARG, "table index %u out of range", h_index[base + c]);
        enc.symbol(h_symbols[base + c], h_center[base + c], h_index[base + c]);
      }
    }
  enc.finish();
  *out_bytes = enc.bytes();
  if (enc.overflow()) return fail(PSWA_E_ARG, "output capacity %zu < %zu bytes", cap, enc.bytes());
  return PSWA_OK;
}

}  // extern "C"
