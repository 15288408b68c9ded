// Internal interfaces between the C ABI / runtime (pswa_capi.cpp), the HIP
// kernels (kernels_*.hip) and the host entropy coder (coder.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace pswa {

// ------------------------------------------------------------- profiling
// Role of a launch, for the live kernel timer (profile.cpp).
enum Role {
  R_ACC_Q, R_ACC_ATTN, R_ACC_O, R_QKV, R_ATTN, R_O, R_GATEUP, R_DOWN, R_HEAD1, R_HEAD2,
  R_EMBED, R_ACCKV, R_BITS, R_GATHER, R_HYPER, R_TKV, R_SUM, R_OTHER, R_PERSIST, R_COUNT
};
const char* role_name(int r);
bool prof_on();
int prof_begin(hipStream_t s);  // -1 when timing is off
void prof_end(int ev, hipStream_t s, int role, double bytes, double flops);

// ------------------------------------------------------------------ GEMM
// Y[m][n] = epilogue( sum_k A[m][k] * W[n][k] ), accumulated k = 0..K-1 in
// order by one thread per output, so a row's value never depends on how many
// rows are in the launch or how they are tiled.
enum AKind { A_FLOAT = 0, A_INT = 1 };
// Arithmetic of a GEMM: FP32 SIMT, or BF16 / FP8 (OCP e4m3fn) MFMA.
constexpr int PSWA_PREC_F32 = 0, PSWA_PREC_BF16 = 1, PSWA_PREC_FP8 = 2;
enum Epi {
  EPI_STORE = 0,   // Y[yrow(m)][n] = acc
  EPI_RESID = 1,   // Y[yrow(m)][n] = R[rrow(m)][n] + acc
  EPI_QKV = 2,     // n < nsplit: Y[m][n] = acc; else Y2[y2row(m)][n - nsplit] = acc
  EPI_SILU = 3,    // Y[yrow(m)][n] = silu(acc)
  EPI_SWIGLU = 4,  // Y[yrow(m)][n] = silu(acc(W)) * acc(W2)
  EPI_HEAD = 5     // mean/scale/centre/index from acc(W) (mean) and acc(W2) (scale)
};

struct HeadOut {
  const float *gmu, *bmu, *gsig, *bsig;  // [C]
  float ln_smin, ln_smax, inv_delta;
  int ldo, col0;                         // output (row, n) at yrow(row) * ldo + col0 + n
                                         // (the column also indexes gmu .. bsig)
  float *mean, *scale;                   // [HW][ldo] rows yrow(m)
  int32_t* center;                       // [HW][C]
  uint16_t* index;                       // [HW][C]
  int32_t* center_c;                     // compact [M][C] copies (or null)
  uint16_t* index_c;
  int* flag;                             // set to 1 on a non-finite mean/scale
  // optional (persistent decode): gather the row's symbols and their bits in
  // the same epilogue; ydec[yrow(m)][n] = ysrc[(src_compact ? m : yrow(m))][n]
  const int32_t* ysrc;
  int src_compact;
  int32_t* ydec;                         // null: no symbols in the epilogue
  float* bits;                           // [HW][C] rows yrow(m)
};

struct GemmArgs {
  int M, N, K;
  int role = R_OTHER;
  const float* X = nullptr;              // A_FLOAT: row m at X + xrow(m)*ldx
  const int32_t* Xi = nullptr;           // A_INT:   row m at Xi + xrow(m)*ldx, times xscale[k]
  const float* xscale = nullptr;
  int ldx = 0;
  const int* xrow = nullptr;             // null: identity
  const float* gain = nullptr;           // RMSNorm prologue gain (null: none)
  const float* W = nullptr;              // [N][K]
  const float* W2 = nullptr;             // paired epilogues: second [N][K]
  int prec = 0;                          // PSWA_PREC_*; low precision reads Wq / W2q
  const void* Wq = nullptr;              // [N][K] BF16 or FP8 copy of W
  const void* W2q = nullptr;
  float wscale = 1.f, w2scale = 1.f;     // 1 / (weight quantization scale)
  // FP8 activations: ascale > 0 is the static per-tensor scale 448 / amax of
  // this projection's input (the RMSNorm output for normed inputs), applied
  // before rounding and divided out after the product; 0 scales each row by
  // 448 / its own maximum.
  float ascale = 0.f;
  // Calibration (FP32 tiles only): when set, the largest |input| this
  // projection multiplies is max-combined into *amax.
  float* amax = nullptr;
  float* Y = nullptr;
  int ldy = 0;
  const int* yrow = nullptr;
  const float* R = nullptr;
  int ldr = 0;
  const int* rrow = nullptr;
  float* Y2 = nullptr;
  int ldy2 = 0;
  const int* y2row = nullptr;
  int nsplit = 0;
  // EPI_STORE's Y, or EPI_QKV's Y2, is a key/value cache stored in BF16
  // (element offsets as for FP32; the buffer's FP32 layout is half used)
  int kv16 = 0;
  HeadOut head{};
};

void gemm_run(AKind ak, bool rms, Epi epi, const GemmArgs& a, hipStream_t s);
double gemm_alg_bytes(const GemmArgs& a, Epi epi);

// Kernels whose dynamic LDS can exceed 64 KiB opt in to 156 KiB (the
// 160 KiB per workgroup less room for their static LDS).
constexpr size_t kMaxDynLds = 156 * 1024;
bool allow_big_lds(const void* fn);

// ------------------------------------------------------------- attention
// A frame in the global position space of a launch: its grid, the global
// index of its position (0, 0), and whether it has previous-frame keys.
struct FrameInfo {
  int H, W, off, n_prev;
};

struct AttnArgs {
  int role;
  int M;                       // query rows
  const int* pos;              // global position of row m (null: m)
  const int* fid;              // frame of row m (null: every row is frame0)
  const FrameInfo* frames;     // frame table indexed by fid
  FrameInfo frame0;
  int HWt;                     // positions in the global space (temporal K/V stride)
  int r, heads, dh, d;
  const float* q; int ldq;     // query row m at q + qrow(m) * ldq
  const int* qrow;             // null: m
  const float* kv;             // [HWt][2d]: K then V per position
  const float* tkv;            // [2][HWt][2d] temporal K/V (or null)
  int kv16;                    // kv and tkv hold BF16 (element offsets as for FP32)
  const float* bias; int nbias;  // [heads][nbias]
  const float* knull;          // accumulator null slot (null in layer mode): its key and value
                               // are read from row HWt of kv (both attention forms)
  const float* vnull;
  int include_self;            // layer mode: the query's own key
  int cycle;                   // 0: causal half-window; c: full window, masked by
                               // step (i + j) mod c (< for the accumulator, <= for layers)
  float* out; int ldo;         // [M][d]
};
// Key slots an attention row scans: spatial window (+ self), null, temporal.
__host__ __device__ inline int attn_slots(const AttnArgs& a) {
  const int k1 = 2 * a.r + 1;
  const int sp = a.cycle ? k1 * k1 : 2 * a.r * (a.r + 1) + (a.include_self ? 1 : 0);
  return sp + (a.knull ? 1 : 0) + (a.tkv ? 2 * k1 * k1 : 0);
}
void attention_f32(const AttnArgs& a, hipStream_t s);
// Row `row` of an accumulator K/V cache [.][2d] := the null key and value
// (BF16 when kv16): the accumulator reads its null slot there.
void null_row(float* acc_kv, size_t row, const float* knull, const float* vnull, int d, int kv16,
              hipStream_t s);
double attn_alg_bytes(const AttnArgs& a);

// ----------------------------------------------------------------- misc
void hyper_embed(const int32_t* z, int Hh, int Wh, int Ch, const float* Wh_, const float* P4,
                 int H, int W, int d, float* h, hipStream_t s);
// ydec[pos(m)][c] = src[(compact ? m : pos(m))][c] for c in [c0, c0 + nc)
void gather_symbols(const int32_t* src, int compact, const int* pos, int M, int C,
                    int32_t* ydec, hipStream_t s, int c0 = 0, int nc = -1);
// Y[m][col0 + k] = RMSNorm of X[m][col0 .. col0 + K) times gain[col0 + k]
// (one channel group's slice normalized on its own), rows m < M
void group_rmsnorm(const float* X, int ldx, int M, int K, int col0, const float* gain, float* Y,
                   int ldy, hipStream_t s);
// bits[pos(m)][c] = -log2(max(P, 1e-9)) of ydec under N(mean, scale)
void symbol_bits(const int* pos, int M, int C, const int32_t* ydec, const float* mean,
                 const float* scale, float* bits, hipStream_t s);
// out[0] = sum of v[0..n) (fixed order, float32 with compensation)
void sum_f32(const float* v, size_t n, float* out, hipStream_t s);
void cdf_select(const float* mean, const float* lsig, size_t n, float ln_smin,
                float inv_delta, int32_t* center, uint16_t* index, hipStream_t s);

// -------------------------------------------------------- entropy coder
constexpr int kScales = 64;
constexpr int kPhases = 16;
constexpr int kTables = kScales * kPhases;
constexpr int kPrecBits = 16;
constexpr double kSigmaMin = 0.11;
constexpr double kSigmaMax = 64.0;

struct CdfTables {
  std::vector<uint32_t> radius;  // [kTables]
  std::vector<uint32_t> offset;  // [kTables + 1] into freq / cum (cum has +1 per table)
  std::vector<uint16_t> freq;    // frequencies
  std::vector<uint32_t> cum_off; // [kTables] offset into cum
  std::vector<uint32_t> cum;     // cumulative, 2R+3 entries per table
};
const CdfTables& cdf_tables();
float ln_sigma_min_f32();
float inv_delta_f32();

class RangeEncoder {
 public:
  RangeEncoder(uint8_t* out, size_t cap) : out_(out), cap_(cap) {}
  void encode(uint32_t start, uint32_t size);
  void bit(uint32_t b);
  void symbol(int32_t v, int32_t center, uint16_t index);
  void finish();
  size_t bytes() const { return n_; }
  bool overflow() const { return overflow_; }

 private:
  void shift_low();
  void put(uint8_t b);
  uint8_t* out_;
  size_t cap_, n_ = 0;
  bool overflow_ = false;
  uint64_t low_ = 0;
  uint32_t range_ = 0xFFFFFFFFu;
  uint8_t cache_ = 0;
  uint64_t cache_size_ = 1;
};

class RangeDecoder {
 public:
  RangeDecoder(const uint8_t* in, size_t n);
  // false on a corrupt or truncated stream
  bool symbol(int32_t center, uint16_t index, int32_t* v);
  bool ok() const { return ok_; }

 private:
  uint32_t next();
  bool bit(uint32_t* b);
  const uint8_t* in_;
  size_t n_, p_ = 0;
  uint32_t range_ = 0xFFFFFFFFu, code_ = 0;
  bool ok_ = true;
  size_t overrun_ = 0;
};

}  // namespace pswa
