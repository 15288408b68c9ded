// Distillation training of a student context model, FP32, hand-written
// kernels (C ABI in include/pswa.h).
//
// One step on a batch of B crops (each its own frame, I- or P-frames):
// forward in the parallel form with every intermediate kept, the loss
// mean((mu - mu_t)^2) + mean((lsig - lsig_t)^2) over all symbols, the
// backward pass of every operation, and AdamW. The forward is the same
// definition as the inference path (Sec. 3.1: hyperprior token, accumulator
// cross-attention over the strictly-past window plus a null slot, pre-norm
// layers with windowed self-attention over the causal window and, for
// P-frames, the windows of two previous frames, SwiGLU MLP, 2-layer head).
//
// Kernels: a tiled FP32 GEMM (three operand layouts, split-K with a
// fixed-order reduction for the weight gradients), row RMSNorm forward and
// backward, window attention forward (log-sum-exp kept) and backward in two
// passes -- per query (dq, softmax and logit gradients per slot) and per key
// (dk, dv gathered over the queries whose window holds the key, in slot
// order), so no atomics are used and every gradient is reproducible --, a
// two-stage column sum for gains, biases and slot biases, elementwise SiLU /
// SwiGLU, the loss with its gradient, and AdamW.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "../../include/pswa.h"
#include "runtime.h"

namespace pswa {
namespace {

constexpr int kT = 256;
constexpr float kRmsEps = 1e-5f;

inline int cdiv(long a, long b) { return int((a + b - 1) / b); }

// ---------------------------------------------------------------- GEMM
// C[m][n] = sum_k A(m, k) B(n, k) (+ beta C), A(m, k) = TA ? A[k*lda + m] :
// A[m*lda + k], B(n, k) = TB ? B[k*ldb + n] : B[n*ldb + k]. 64x64 tiles,
// 16-deep k slices staged in LDS, 4x4 outputs per thread. With gridDim.z > 1
// block z covers k in [z*kc, (z+1)*kc) and writes its partial sum to
// C + z*M*N (ldc = N); k_splitk_reduce adds the partials in order.
template <bool TA, bool TB>
__global__ void __launch_bounds__(kT) k_tgemm(int M, int N, int K, const float* __restrict__ A,
                                              int lda, const float* __restrict__ B, int ldb,
                                              float* C, int ldc, float beta, int kc) {
  __shared__ float As[16][68];
  __shared__ float Bs[16][68];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int kb = blockIdx.z * kc, ke = min(K, kb + kc);
  float acc[4][4] = {};
  for (int k0 = kb; k0 < ke; k0 += 16) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!TA) {
        const int m = tid >> 2, k = (tid & 3) * 4 + u;
        const int gm = m0 + m, gk = k0 + k;
        As[k][m] = (gm < M && gk < ke) ? A[(size_t)gm * lda + gk] : 0.f;
      } else {
        const int k = tid >> 4, m = (tid & 15) * 4 + u;
        const int gm = m0 + m, gk = k0 + k;
        As[k][m] = (gm < M && gk < ke) ? A[(size_t)gk * lda + gm] : 0.f;
      }
      if (!TB) {
        const int n = tid >> 2, k = (tid & 3) * 4 + u;
        const int gn = n0 + n, gk = k0 + k;
        Bs[k][n] = (gn < N && gk < ke) ? B[(size_t)gn * ldb + gk] : 0.f;
      } else {
        const int k = tid >> 4, n = (tid & 15) * 4 + u;
        const int gn = n0 + n, gk = k0 + k;
        Bs[k][n] = (gn < N && gk < ke) ? B[(size_t)gk * ldb + gn] : 0.f;
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[k][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[k][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
  const bool split = gridDim.z > 1;
  float* Cz = split ? C + (size_t)blockIdx.z * M * N : C;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + ty * 4 + i;
    if (m >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + tx * 4 + j;
      if (n >= N) continue;
      if (split) {
        Cz[(size_t)m * N + n] = acc[i][j];
      } else {
        float* c = C + (size_t)m * ldc + n;
        *c = beta != 0.f ? acc[i][j] + beta * *c : acc[i][j];
      }
    }
  }
}

__global__ void k_splitk_reduce(const float* part, int splits, int M, int N, float* C, int ldc,
                                float beta) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)M * N) return;
  const int m = idx / N, n = idx % N;
  float s = 0.f;
  for (int z = 0; z < splits; ++z) s += part[(size_t)z * M * N + idx];
  float* c = C + (size_t)m * ldc + n;
  *c = beta != 0.f ? s + beta * *c : s;
}

// ------------------------------------------------------------- RMSNorm
// One wave per row. Forward: Y = X * rstd * g. Backward (with c = sum_k
// dY_k g_k X_k): dX = base + rstd g dY - X rstd^3 c / K, and P = dY X rstd
// (the per-row terms of the gain gradient).
__device__ __forceinline__ float wsum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ void k_rms_fwd(const float* X, int ldx, const float* g, float* Y, int ldy, float* rstd,
                          int rows, int K) {
  const int row = blockIdx.x * (kT / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= rows) return;
  const float* x = X + (size_t)row * ldx;
  float ss = 0.f;
  for (int c = lane; c < K; c += 64) ss = fmaf(x[c], x[c], ss);
  ss = wsum(ss);
  const float r = 1.0f / sqrtf(ss / float(K) + kRmsEps);
  if (lane == 0) rstd[row] = r;
  for (int c = lane; c < K; c += 64) Y[(size_t)row * ldy + c] = x[c] * r * g[c];
}

__global__ void k_rms_bwd(const float* X, int ldx, const float* g, const float* rstd,
                          const float* dY, int lddy, const float* base, int ldb, float* dX,
                          int lddx, float* P, int rows, int K) {
  const int row = blockIdx.x * (kT / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= rows) return;
  const float* x = X + (size_t)row * ldx;
  const float* dy = dY + (size_t)row * lddy;
  const float r = rstd[row];
  float c = 0.f;
  for (int k = lane; k < K; k += 64) c = fmaf(dy[k] * g[k], x[k], c);
  c = wsum(c);
  const float r3c = r * r * r * c / float(K);
  for (int k = lane; k < K; k += 64) {
    float v = r * g[k] * dy[k] - x[k] * r3c;
    if (base) v += base[(size_t)row * ldb + k];
    dX[(size_t)row * lddx + k] = v;
    P[(size_t)row * K + k] = dy[k] * x[k] * r;
  }
}

// ------------------------------------------------------- column sums
// part[chunk][c] = sum of X[rows of chunk][c]; out[c] (+)= sum_chunk part.
__global__ void k_colsum_part(const float* X, int ldx, int rows, int K, int chunk, float* part) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= K) return;
  const int r0 = blockIdx.y * chunk, r1 = min(rows, r0 + chunk);
  float s = 0.f;
  for (int r = r0; r < r1; ++r) s += X[(size_t)r * ldx + c];
  part[(size_t)blockIdx.y * K + c] = s;
}

__global__ void k_colsum_final(const float* part, int nchunk, int K, float* out, int add) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= K) return;
  float s = 0.f;
  for (int z = 0; z < nchunk; ++z) s += part[(size_t)z * K + c];
  out[c] = add ? out[c] + s : s;
}

// dst[h][s] += src[h][s] for s < n (slot-bias gradients into their tensor)
__global__ void k_add_strided(const float* src, int heads, int Ssrc, int n, float* dst, int Sdst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= heads * n) return;
  const int h = i / n, s = i % n;
  dst[h * Sdst + s] += src[h * Ssrc + s];
}

// --------------------------------------------------------- elementwise
__global__ void k_to_float(const int32_t* y, const float* g, float* yf, float* yg, long n, int C) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float v = float(y[i]);
  if (yf) yf[i] = v;
  if (yg) yg[i] = v * g[i % C];
}

__device__ __forceinline__ float sigm(float x) { return 1.0f / (1.0f + expf(-x)); }

__global__ void k_swiglu_fwd(const float* G, const float* U, float* Hm, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) Hm[i] = G[i] * sigm(G[i]) * U[i];
}

__global__ void k_swiglu_bwd(const float* G, const float* U, const float* dHm, float* dG,
                             float* dU, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = G[i], s = sigm(g), si = g * s;
  dG[i] = dHm[i] * U[i] * s * (1.0f + g * (1.0f - s));
  dU[i] = dHm[i] * si;
}

__global__ void k_silu_fwd(const float* T, float* S, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) S[i] = T[i] * sigm(T[i]);
}

__global__ void k_silu_bwd(const float* T, const float* dS, float* dT, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float t = T[i], s = sigm(t);
  dT[i] = dS[i] * s * (1.0f + t * (1.0f - s));
}

__global__ void k_mul(const float* a, const float* b, float* out, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] * b[i];
}

__global__ void k_fill(float* p, long n, float v) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ------------------------------------------------------------ head loss
// Per symbol: mu = gmu t1 + bmu, raw = gsig t2 + bsig, ls = clamp(raw);
// loss terms (mu - mu_t)^2 + (ls - ls_t)^2, gradients scaled by 2 / n.
__global__ void k_head_loss(const float* T, int rows, int C, const float* gmu, const float* bmu,
                            const float* gsig, const float* bsig, const float* mu_t,
                            const float* ls_t, float ln_min, float ln_max, float two_over_n,
                            float* dT, float* Pgm, float* Pbm, float* Pgs, float* Pbs,
                            float* loss_part) {
  __shared__ float red[kT];
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.f;
  if (i < (long)rows * C) {
    const int row = i / C, c = i % C;
    const float t1 = T[(size_t)row * 2 * C + c], t2 = T[(size_t)row * 2 * C + C + c];
    const float mu = gmu[c] * t1 + bmu[c];
    const float raw = gsig[c] * t2 + bsig[c];
    const float ls = fminf(ln_max, fmaxf(ln_min, raw));
    const float em = mu - mu_t[i], es = ls - ls_t[i];
    l = em * em + es * es;
    const float dmu = two_over_n * em;
    const float dls = (raw >= ln_min && raw <= ln_max) ? two_over_n * es : 0.f;
    dT[(size_t)row * 2 * C + c] = dmu * gmu[c];
    dT[(size_t)row * 2 * C + C + c] = dls * gsig[c];
    Pgm[i] = dmu * t1;
    Pbm[i] = dmu;
    Pgs[i] = dls * t2;
    Pbs[i] = dls;
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// ----------------------------------------------------- hyperprior token
// dP4[sub][n] = sum of dH over positions with that sub-position;
// dHc[cell][n] = sum of dH over the cell's positions (then dW_h = dHc^T z).
__global__ void k_hyper_p4_grad(const float* dH, int B, int H, int W, int d, float* dP4) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 16 * d) return;
  const int sub = i / d, n = i % d, a = sub / 4, bb = sub % 4;
  float s = 0.f;
  for (int b = 0; b < B; ++b)
    for (int ii = a; ii < H; ii += 4)
      for (int jj = bb; jj < W; jj += 4) s += dH[((size_t)b * H * W + ii * W + jj) * d + n];
  dP4[i] += s;
}

__global__ void k_hyper_cell_sum(const float* dH, int B, int H, int W, int Hh, int Wh, int d,
                                 float* dHc) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)B * Hh * Wh * d) return;
  const int n = i % d;
  const long cell = i / d;
  const int b = cell / (Hh * Wh), ci = (cell % (Hh * Wh)) / Wh, cj = cell % Wh;
  float s = 0.f;
  for (int a = 0; a < 4 && 4 * ci + a < H; ++a)
    for (int bb = 0; bb < 4 && 4 * cj + bb < W; ++bb)
      s += dH[((size_t)b * H * W + (4 * ci + a) * W + 4 * cj + bb) * d + n];
  dHc[i] = s;
}

// ------------------------------------------------------------ attention
// Slots of query p = (i, j) in crop b, in bias-slot order:
//   s < nc (nc = 2r(r+1)): the causal window (r rows above, columns -r..r,
//     then r cells to the left);
//   s == nc: the null slot (accumulator) or p itself (layers);
//   s = ns + t (layers of P-frames, ns = nc + 1): previous frame tau =
//     t / (2r+1)^2 + 1 at offset (t mod (2r+1)^2) in a (2r+1)^2 window.
struct TAttn {
  int N, HW, H, W, heads, r, acc;  // acc: accumulator (null slot), else layer
  int S;                           // slots (buffer stride)
  const float* Q;
  int ldq;
  const float *K, *V;              // spatial keys of the same rows
  int ldk;
  const float *Kt, *Vt;            // temporal keys, rows (b*2 + tau-1)*HW + pos (or null)
  int ldt;
  const float *knull, *vnull;
  const float* bias;               // [heads][nbias]
  int nbias;
  const float* O;                  // attention output (backward)
  const float* dO;
  int ldo;
};

__device__ __forceinline__ void slot_offset(int s, int r, int* a, int* b) {
  const int k1 = 2 * r + 1;
  if (s < r * k1) {
    *a = -r + s / k1;
    *b = -r + s % k1;
  } else {
    *a = 0;
    *b = -r + (s - r * k1);
  }
}

// Key row (or -1) and bias of slot s for query row p; kind 0 spatial, 1
// temporal, 2 null.
__device__ __forceinline__ int slot_key(const TAttn& A, int p, int s, int* kind) {
  const int nc = 2 * A.r * (A.r + 1);
  const int b = p / A.HW, pos = p % A.HW, i = pos / A.W, j = pos % A.W;
  if (s < nc) {
    int a, bb;
    slot_offset(s, A.r, &a, &bb);
    *kind = 0;
    const int ii = i + a, jj = j + bb;
    return (ii >= 0 && ii < A.H && jj >= 0 && jj < A.W) ? b * A.HW + ii * A.W + jj : -1;
  }
  if (s == nc) {
    *kind = A.acc ? 2 : 0;
    return p;
  }
  const int k1 = 2 * A.r + 1, t = s - nc - 1, tau = t / (k1 * k1), rem = t % (k1 * k1);
  const int ii = i - A.r + rem / k1, jj = j - A.r + rem % k1;
  *kind = 1;
  return (ii >= 0 && ii < A.H && jj >= 0 && jj < A.W) ? (b * 2 + tau) * A.HW + ii * A.W + jj : -1;
}

__device__ __forceinline__ float slot_bias(const TAttn& A, int h, int s) {
  const int nc = 2 * A.r * (A.r + 1);
  if (A.acc && s == nc) return 0.f;
  return A.bias[h * A.nbias + s];
}

template <int DH>
__device__ __forceinline__ void key_rows(const TAttn& A, int kind, int row, int h,
                                         const float** k, const float** v) {
  if (kind == 0) {
    *k = A.K + (size_t)row * A.ldk + h * DH;
    *v = A.V + (size_t)row * A.ldk + h * DH;
  } else if (kind == 1) {
    *k = A.Kt + (size_t)row * A.ldt + h * DH;
    *v = A.Vt + (size_t)row * A.ldt + h * DH;
  } else {
    *k = A.knull + h * DH;
    *v = A.vnull + h * DH;
  }
}

// forward: thread per (row, head); online softmax over the slots
template <int DH>
__global__ void __launch_bounds__(128) k_tattn_fwd(TAttn A, float* Out, int ldout, float* lse) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)A.N * A.heads) return;
  const int p = idx / A.heads, h = idx % A.heads;
  const float scale = 1.0f / sqrtf(float(DH));
  float q[DH], o[DH];
  const float* qp = A.Q + (size_t)p * A.ldq + h * DH;
#pragma unroll
  for (int c = 0; c < DH; ++c) {
    q[c] = qp[c];
    o[c] = 0.f;
  }
  float m = -INFINITY, l = 0.f;
  for (int s = 0; s < A.S; ++s) {
    int kind;
    const int row = slot_key(A, p, s, &kind);
    if (row < 0) continue;
    const float *k, *v;
    key_rows<DH>(A, kind, row, h, &k, &v);
    float dot = 0.f;
#pragma unroll
    for (int c = 0; c < DH; ++c) dot = fmaf(q[c], k[c], dot);
    const float lg = dot * scale + slot_bias(A, h, s);
    const float mn = fmaxf(m, lg);
    const float corr = expf(m - mn), w = expf(lg - mn);
    l = l * corr + w;
#pragma unroll
    for (int c = 0; c < DH; ++c) o[c] = o[c] * corr + w * v[c];
    m = mn;
  }
  float* op = Out + (size_t)p * ldout + h * DH;
#pragma unroll
  for (int c = 0; c < DH; ++c) op[c] = o[c] / l;
  lse[idx] = m + logf(l);
}

// backward, query side: P_s, dS_s = P_s (dO.V_s - dO.O) per slot; dq
template <int DH>
__global__ void __launch_bounds__(128) k_tattn_bwd_q(TAttn A, const float* lse, float* dQ, int lddq, float* Pbuf,
                              float* dSbuf) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)A.N * A.heads) return;
  const int p = idx / A.heads, h = idx % A.heads;
  const float scale = 1.0f / sqrtf(float(DH));
  float q[DH], go[DH], dq[DH];
  const float* qp = A.Q + (size_t)p * A.ldq + h * DH;
  const float* gp = A.dO + (size_t)p * A.ldo + h * DH;
  const float* op = A.O + (size_t)p * A.ldo + h * DH;
  float D = 0.f;
#pragma unroll
  for (int c = 0; c < DH; ++c) {
    q[c] = qp[c];
    go[c] = gp[c];
    dq[c] = 0.f;
    D = fmaf(go[c], op[c], D);
  }
  const float L = lse[idx];
  float* pb = Pbuf + idx * A.S;
  float* sb = dSbuf + idx * A.S;
  for (int s = 0; s < A.S; ++s) {
    int kind;
    const int row = slot_key(A, p, s, &kind);
    if (row < 0) {
      pb[s] = 0.f;
      sb[s] = 0.f;
      continue;
    }
    const float *k, *v;
    key_rows<DH>(A, kind, row, h, &k, &v);
    float dot = 0.f, dp = 0.f;
#pragma unroll
    for (int c = 0; c < DH; ++c) {
      dot = fmaf(q[c], k[c], dot);
      dp = fmaf(go[c], v[c], dp);
    }
    const float P = expf(dot * scale + slot_bias(A, h, s) - L);
    const float dS = P * (dp - D);
    pb[s] = P;
    sb[s] = dS;
#pragma unroll
    for (int c = 0; c < DH; ++c) dq[c] = fmaf(dS * scale, k[c], dq[c]);
  }
  float* dqp = dQ + (size_t)p * lddq + h * DH;
#pragma unroll
  for (int c = 0; c < DH; ++c) dqp[c] = dq[c];
}

// backward, key side (spatial keys): thread per (key row, head); the
// queries whose slot s holds key (i, j) sit at (i, j) - offset(s)
template <int DH>
__global__ void __launch_bounds__(128) k_tattn_bwd_kv(TAttn A, const float* Pbuf, const float* dSbuf, float* dK,
                               float* dV, int lddk) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)A.N * A.heads) return;
  const int kr = idx / A.heads, h = idx % A.heads;
  const int b = kr / A.HW, pos = kr % A.HW, i = pos / A.W, j = pos % A.W;
  const float scale = 1.0f / sqrtf(float(DH));
  const int nc = 2 * A.r * (A.r + 1);
  const int nsp = A.acc ? nc : nc + 1;  // spatial slots (self included for layers)
  float dk[DH], dv[DH];
#pragma unroll
  for (int c = 0; c < DH; ++c) dk[c] = dv[c] = 0.f;
  for (int s = 0; s < nsp; ++s) {
    int a = 0, bb = 0;
    if (s < nc) slot_offset(s, A.r, &a, &bb);
    const int ii = i - a, jj = j - bb;
    if (ii < 0 || ii >= A.H || jj < 0 || jj >= A.W) continue;
    const int p = b * A.HW + ii * A.W + jj;
    const long pi = (long)p * A.heads + h;
    const float ds = dSbuf[pi * A.S + s] * scale, P = Pbuf[pi * A.S + s];
    const float* qp = A.Q + (size_t)p * A.ldq + h * DH;
    const float* gp = A.dO + (size_t)p * A.ldo + h * DH;
#pragma unroll
    for (int c = 0; c < DH; ++c) {
      dk[c] = fmaf(ds, qp[c], dk[c]);
      dv[c] = fmaf(P, gp[c], dv[c]);
    }
  }
  float* kp = dK + (size_t)kr * lddk + h * DH;
  float* vp = dV + (size_t)kr * lddk + h * DH;
#pragma unroll
  for (int c = 0; c < DH; ++c) {
    kp[c] = dk[c];
    vp[c] = dv[c];
  }
}

// backward, temporal keys: thread per (previous-frame row, head)
template <int DH>
__global__ void __launch_bounds__(128) k_tattn_bwd_tkv(TAttn A, const float* Pbuf, const float* dSbuf, float* dK,
                                float* dV, int lddk) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)2 * A.N * A.heads) return;
  const int kr = idx / A.heads, h = idx % A.heads;
  const int bt = kr / A.HW, b = bt / 2, tau = bt % 2;
  const int pos = kr % A.HW, i = pos / A.W, j = pos % A.W;
  const float scale = 1.0f / sqrtf(float(DH));
  const int k1 = 2 * A.r + 1, ns = 2 * A.r * (A.r + 1) + 1;
  float dk[DH], dv[DH];
#pragma unroll
  for (int c = 0; c < DH; ++c) dk[c] = dv[c] = 0.f;
  for (int t = 0; t < k1 * k1; ++t) {
    const int a = -A.r + t / k1, bb = -A.r + t % k1;
    const int ii = i - a, jj = j - bb;
    if (ii < 0 || ii >= A.H || jj < 0 || jj >= A.W) continue;
    const int p = b * A.HW + ii * A.W + jj;
    const long pi = (long)p * A.heads + h;
    const int s = ns + tau * k1 * k1 + t;
    const float ds = dSbuf[pi * A.S + s] * scale, P = Pbuf[pi * A.S + s];
    const float* qp = A.Q + (size_t)p * A.ldq + h * DH;
    const float* gp = A.dO + (size_t)p * A.ldo + h * DH;
#pragma unroll
    for (int c = 0; c < DH; ++c) {
      dk[c] = fmaf(ds, qp[c], dk[c]);
      dv[c] = fmaf(P, gp[c], dv[c]);
    }
  }
  float* kp = dK + (size_t)kr * lddk + h * DH;
  float* vp = dV + (size_t)kr * lddk + h * DH;
#pragma unroll
  for (int c = 0; c < DH; ++c) {
    kp[c] = dk[c];
    vp[c] = dv[c];
  }
}

// null key/value gradients: column partials over row chunks of
// dS(null) * Q * scale and P(null) * dO
__global__ void k_null_part(const float* Pbuf, const float* dSbuf, int S, int slot,
                            const float* Q, int ldq, const float* dO, int ldo, int rows, int d,
                            int dh, int heads, float scale, int chunk, float* part) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= 2 * d) return;
  const bool isv = c >= d;
  const int cc = isv ? c - d : c, h = cc / dh;
  const int r0 = blockIdx.y * chunk, r1 = min(rows, r0 + chunk);
  float s = 0.f;
  for (int r = r0; r < r1; ++r) {
    const long pi = ((long)r * heads + h) * S + slot;
    s += isv ? Pbuf[pi] * dO[(size_t)r * ldo + cc] : dSbuf[pi] * scale * Q[(size_t)r * ldq + cc];
  }
  part[(size_t)blockIdx.y * 2 * d + c] = s;
}

// ---------------------------------------------------------------- AdamW
__global__ void k_adamw(float* w, const float* g, float* m, float* v, long n, float lr, float wd,
                        float b1, float b2, float eps, float c1, float c2) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / c1, vh = vi / c2;
  float wi = w[i];
  if (wd != 0.f) wi = wi * (1.0f - lr * wd);
  w[i] = wi - lr * mh / (sqrtf(vh) + eps);
}

}  // namespace
}  // namespace pswa

using namespace pswa;

// ==================================================================== host
namespace {

constexpr size_t kTAlign = 64;  // floats per tensor alignment in the trainer

struct Lay {  // per-layer forward state
  float *x, *u, *r1, *qkv, *up, *rp, *tkv, *att, *lse, *y, *v, *r2, *g, *upr, *hm;
};

}  // namespace

struct pswa_trainer {
  pswa_model_desc desc{};
  NetDims x{};
  int Bmax = 0, H = 0, W = 0, Hh = 0, Wh = 0;
  long N = 0;  // rows of a full batch
  std::vector<std::pair<size_t, size_t>> span;  // (offset, floats) per tensor, padded
  std::vector<std::pair<size_t, size_t>> span_blob;  // the same in the host blob
  size_t nparam = 0, blob_floats = 0;
  int step = 0;
  // parameters
  float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  // forward
  float *yf, *yg, *ypf, *ypg, *zf, *h, *e, *ep, *uq, *rq, *Q0, *ukv, *rkv, *KV0, *A0, *lse0;
  std::vector<Lay> lay;  // L + 1 entries: lay[l].x is layer l's input; lay[L].x the output
  float *zh, *rz, *T1, *S1, *T;
  // backward
  float *dX, *dY, *dA, *dQKV, *dU, *dV, *dG, *dUp, *dHm, *dTKV, *dUP, *dEp, *dE, *dKV0, *dQ0, *dH,
      *dHc, *dT, *dS1, *dT1, *dZ, *dYg, *dYpg, *Pg, *Pg2, *Pbuf, *dSbuf, *part, *loss_part,
      *bias_tmp;
  size_t part_cap = 0;
  size_t bytes = 0;
};

namespace {

inline float* T_(pswa_trainer* t, float* base, int k) { return base + t->span[k].first; }

enum {
  I_HW = 0, I_P4, I_ING, I_INW, I_GQ, I_WQ, I_GKV, I_WKV, I_KNULL, I_VNULL, I_ABIAS, I_AWO
};
inline int I_L(int l, int k) { return 12 + 8 * l + k; }  // g1 Wqkv bias Wo g2 Wgate Wup Wdown
inline int I_H(int L, int k) { return 12 + 8 * L + k; }  // g W1 W2 gmu bmu gsig bsig

bool decayed_tensor(int k, int L) {
  if (k == I_HW || k == I_INW || k == I_WQ || k == I_WKV || k == I_AWO) return true;
  if (k >= 12 && k < 12 + 8 * L) {
    const int r = (k - 12) % 8;
    return r == 1 || r == 3 || r == 5 || r == 6 || r == 7;
  }
  return k == I_H(L, 1) || k == I_H(L, 2);
}

void lay_out(pswa_trainer* t, void* base) {
  Layout Lo(base);
  const NetDims& x = t->x;
  const size_t N = t->N, N2 = 2 * N, d = x.d, F = x.F, C = x.C, hd = x.heads;
  const size_t S = x.n_sp + x.n_tm;
  auto f = [&](size_t n) { return Lo.take<float>(n); };
  t->w = f(t->nparam);
  t->g = f(t->nparam);
  t->m = f(t->nparam);
  t->v = f(t->nparam);
  t->yf = f(N * C); t->yg = f(N * C); t->ypf = f(N2 * C); t->ypg = f(N2 * C);
  t->zf = f((size_t)t->Bmax * t->Hh * t->Wh * x.Ch);
  t->h = f(N * d); t->e = f(N * d); t->ep = f(N2 * d);
  t->uq = f(N * d); t->rq = f(N); t->Q0 = f(N * d);
  t->ukv = f(N * d); t->rkv = f(N); t->KV0 = f(N * 2 * d);
  t->A0 = f(N * d); t->lse0 = f(N * hd);
  t->lay.assign(x.L + 1, Lay{});
  for (int l = 0; l <= x.L; ++l) {
    Lay& a = t->lay[l];
    a.x = f(N * d);
    if (l == x.L) break;
    a.u = f(N * d); a.r1 = f(N); a.qkv = f(N * 3 * d);
    a.up = f(N2 * d); a.rp = f(N2); a.tkv = f(N2 * 2 * d);
    a.att = f(N * d); a.lse = f(N * hd); a.y = f(N * d); a.v = f(N * d); a.r2 = f(N);
    a.g = f(N * F); a.upr = f(N * F); a.hm = f(N * F);
  }
  t->zh = f(N * d); t->rz = f(N); t->T1 = f(N * d); t->S1 = f(N * d); t->T = f(N * 2 * C);
  t->dX = f(N * d); t->dY = f(N * d); t->dA = f(N * d); t->dQKV = f(N * 3 * d); t->dU = f(N * d);
  t->dV = f(N * d); t->dG = f(N * F); t->dUp = f(N * F); t->dHm = f(N * F);
  t->dTKV = f(N2 * 2 * d); t->dUP = f(N2 * d); t->dEp = f(N2 * d); t->dE = f(N * d);
  t->dKV0 = f(N * 2 * d); t->dQ0 = f(N * d); t->dH = f(N * d);
  t->dHc = f((size_t)t->Bmax * t->Hh * t->Wh * d);
  t->dT = f(N * 2 * C); t->dS1 = f(N * d); t->dT1 = f(N * d); t->dZ = f(N * d);
  t->dYg = f(N * C); t->dYpg = f(N2 * C);
  t->Pg = f(N2 * std::max(d, C)); t->Pg2 = f(4 * N * C);
  t->Pbuf = f(N * hd * S); t->dSbuf = f(N * hd * S);
  t->part_cap = std::max<size_t>(64 * 2048 * 4, (size_t)64 * 1024 * 1024 / 4);
  t->part = f(t->part_cap);
  t->loss_part = f((N * C + kT - 1) / kT + 64);
  t->bias_tmp = f(hd * S + 64);
  t->bytes = Lo.used;
}

// ---- launch helpers
void gemm(pswa_trainer* t, bool ta, bool tb, int M, int N, int K, const float* A, int lda,
          const float* B, int ldb, float* C, int ldc, float beta, hipStream_t s) {
  if (M <= 0 || N <= 0 || K <= 0) return;
  const int tiles = cdiv(M, 64) * cdiv(N, 64);
  int splits = 1;
  if (tiles < 128 && K >= 4096) {
    splits = std::min(cdiv(K, 1024), 64);
    while (splits > 1 && (size_t)splits * M * N > t->part_cap) --splits;
  }
  const int kc = cdiv(cdiv(K, splits), 16) * 16;
  splits = cdiv(K, kc);
  dim3 grid(cdiv(N, 64), cdiv(M, 64), splits);
  float* out = splits > 1 ? t->part : C;
  const int ldo = splits > 1 ? N : ldc;
#define PSWA_G(TA_, TB_) \
  hipLaunchKernelGGL((k_tgemm<TA_, TB_>), grid, dim3(kT), 0, s, M, N, K, A, lda, B, ldb, out, ldo, beta, kc)
  if (!ta && !tb) PSWA_G(false, false);
  else if (!ta && tb) PSWA_G(false, true);
  else if (ta && !tb) PSWA_G(true, false);
  else PSWA_G(true, true);
#undef PSWA_G
  if (splits > 1)
    hipLaunchKernelGGL(k_splitk_reduce, dim3(cdiv((long)M * N, kT)), dim3(kT), 0, s, t->part,
                       splits, M, N, C, ldc, beta);
}

// Y[rows][out] (+)= X[rows][in] W[out][in]^T
void lin(pswa_trainer* t, int rows, int out, int in, const float* X, int ldx, const float* W,
         float* Y, int ldy, float beta, hipStream_t s) {
  gemm(t, false, false, rows, out, in, X, ldx, W, in, Y, ldy, beta, s);
}
// dX[rows][in] (+)= dY[rows][out] W[out][in]
void lin_dx(pswa_trainer* t, int rows, int out, int in, const float* dY, int lddy, const float* W,
            float* dX, int lddx, float beta, hipStream_t s) {
  gemm(t, false, true, rows, in, out, dY, lddy, W, in, dX, lddx, beta, s);
}
// dW[out][in] += dY^T X
void lin_dw(pswa_trainer* t, int rows, int out, int in, const float* dY, int lddy,
            const float* X, int ldx, float* dW, hipStream_t s) {
  gemm(t, true, true, out, in, rows, dY, lddy, X, ldx, dW, in, 1.0f, s);
}

void rms_fwd(long rows, int K, const float* X, int ldx, const float* g, float* Y, int ldy,
             float* rstd, hipStream_t s) {
  hipLaunchKernelGGL(k_rms_fwd, dim3(cdiv(rows, kT / 64)), dim3(kT), 0, s, X, ldx, g, Y, ldy,
                     rstd, int(rows), K);
}

void colsum(pswa_trainer* t, const float* X, int ldx, long rows, int K, float* out, bool add,
            hipStream_t s) {
  const int chunk = 256;
  const int nch = cdiv(rows, chunk);
  hipLaunchKernelGGL(k_colsum_part, dim3(cdiv(K, kT), nch), dim3(kT), 0, s, X, ldx, int(rows), K,
                     chunk, t->part);
  hipLaunchKernelGGL(k_colsum_final, dim3(cdiv(K, kT)), dim3(kT), 0, s, t->part, nch, K, out,
                     add ? 1 : 0);
}

// dX = base + RMSNorm backward; gain gradient added to dg
void rms_bwd(pswa_trainer* t, long rows, int K, const float* X, int ldx, const float* gain,
             const float* rstd, const float* dY, int lddy, const float* base, int ldb, float* dX,
             int lddx, float* dg, hipStream_t s) {
  hipLaunchKernelGGL(k_rms_bwd, dim3(cdiv(rows, kT / 64)), dim3(kT), 0, s, X, ldx, gain, rstd,
                     dY, lddy, base, ldb, dX, lddx, t->Pg, int(rows), K);
  colsum(t, t->Pg, K, rows, K, dg, true, s);
}

void attn_fwd(const TAttn& A, int dh, float* out, int ldout, float* lse, hipStream_t s) {
  const dim3 g(cdiv((long)A.N * A.heads, 128)), b(128);
  switch (dh) {
    case 16: hipLaunchKernelGGL(k_tattn_fwd<16>, g, b, 0, s, A, out, ldout, lse); break;
    case 32: hipLaunchKernelGGL(k_tattn_fwd<32>, g, b, 0, s, A, out, ldout, lse); break;
    case 48: hipLaunchKernelGGL(k_tattn_fwd<48>, g, b, 0, s, A, out, ldout, lse); break;
    default: hipLaunchKernelGGL(k_tattn_fwd<64>, g, b, 0, s, A, out, ldout, lse); break;
  }
}

void attn_bwd(pswa_trainer* t, const TAttn& A, int dh, const float* lse, float* dQ, int lddq,
              float* dK, float* dV, int lddk, float* dKt, float* dVt, int lddt, hipStream_t s) {
  const dim3 g(cdiv((long)A.N * A.heads, 128)), b(128), g2(cdiv(2L * A.N * A.heads, 128));
#define PSWA_AB(D_)                                                                            \
  hipLaunchKernelGGL(k_tattn_bwd_q<D_>, g, b, 0, s, A, lse, dQ, lddq, t->Pbuf, t->dSbuf);      \
  hipLaunchKernelGGL(k_tattn_bwd_kv<D_>, g, b, 0, s, A, t->Pbuf, t->dSbuf, dK, dV, lddk);      \
  if (A.Kt) hipLaunchKernelGGL(k_tattn_bwd_tkv<D_>, g2, b, 0, s, A, t->Pbuf, t->dSbuf, dKt, dVt, lddt);
  switch (dh) {
    case 16: PSWA_AB(16); break;
    case 32: PSWA_AB(32); break;
    case 48: PSWA_AB(48); break;
    default: PSWA_AB(64); break;
  }
#undef PSWA_AB
}

TAttn attn_args(const pswa_trainer* t, int nrows, bool acc, bool temporal) {
  const NetDims& x = t->x;
  TAttn A{};
  A.N = nrows;
  A.HW = t->H * t->W;
  A.H = t->H;
  A.W = t->W;
  A.heads = x.heads;
  A.r = x.r;
  A.acc = acc ? 1 : 0;
  A.S = acc ? x.n_acc + 1 : x.n_sp + (temporal ? x.n_tm : 0);
  return A;
}

}  // namespace

extern "C" {

size_t pswa_train_workspace_bytes(const pswa_model_desc* student, int max_crops, int H, int W) {
  std::string why;
  if (!model_desc_valid(student, &why) || student->prec != PSWA_FP32 || student->cycle != 0 ||
      student->ch_groups != 0)
    return 0;
  if (max_crops < 1 || H < 1 || W < 1 || (long)max_crops * H * W > (1L << 22)) return 0;
  pswa_trainer t;
  t.desc = *student;
  t.x = model_dims(*student);
  t.Bmax = max_crops;
  t.H = H;
  t.W = W;
  t.Hh = (H + 3) / 4;
  t.Wh = (W + 3) / 4;
  t.N = (long)max_crops * H * W;
  t.nparam = model_blob_spans(t.x, kTAlign, &t.span);
  lay_out(&t, nullptr);
  return t.bytes;
}

pswa_status pswa_train_create(const pswa_model_desc* student, const float* h_blob,
                              size_t blob_floats, int max_crops, int H, int W, void* d_ws,
                              size_t ws_bytes, void* stream, pswa_trainer** out) {
  if (!out) return fail(PSWA_E_ARG, "out is null");
  *out = nullptr;
  std::string why;
  if (!model_desc_valid(student, &why))
    return fail(PSWA_E_ARG, "invalid model desc: %s", why.c_str());
  if (student->prec != PSWA_FP32) return fail(PSWA_E_UNSUPPORTED, "training runs in FP32");
  if (student->cycle != 0)
    return fail(PSWA_E_UNSUPPORTED, "training supports the wavefront schedule only");
  if (student->ch_groups != 0)
    return fail(PSWA_E_UNSUPPORTED, "training supports models without channel groups only");
  const size_t need_ws = pswa_train_workspace_bytes(student, max_crops, H, W);
  if (need_ws == 0) return fail(PSWA_E_SHAPE, "invalid crop shape or count");
  if (!h_blob || !d_ws || (reinterpret_cast<uintptr_t>(d_ws) % kAlign) != 0)
    return fail(PSWA_E_ARG, "null blob or unaligned workspace");
  if (ws_bytes < need_ws) return fail(PSWA_E_ARG, "workspace %zu bytes < %zu", ws_bytes, need_ws);
  std::unique_ptr<pswa_trainer> t(new pswa_trainer);
  t->desc = *student;
  t->x = model_dims(*student);
  t->Bmax = max_crops;
  t->H = H;
  t->W = W;
  t->Hh = (H + 3) / 4;
  t->Wh = (W + 3) / 4;
  t->N = (long)max_crops * H * W;
  t->nparam = model_blob_spans(t->x, kTAlign, &t->span);
  t->blob_floats = model_blob_spans(t->x, 1, &t->span_blob);
  if (blob_floats != t->blob_floats)
    return fail(PSWA_E_SHAPE, "blob has %zu floats, model needs %zu", blob_floats, t->blob_floats);
  lay_out(t.get(), d_ws);
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<float> padded(t->nparam, 0.f);
  for (size_t k = 0; k < t->span.size(); ++k)
    std::memcpy(padded.data() + t->span[k].first, h_blob + t->span_blob[k].first,
                t->span[k].second * sizeof(float));
  PSWA_HIP_TRY(hipMemcpyAsync(t->w, padded.data(), t->nparam * sizeof(float),
                              hipMemcpyHostToDevice, s));
  for (float* p : {t->g, t->m, t->v})
    hipLaunchKernelGGL(k_fill, dim3(cdiv(t->nparam, kT)), dim3(kT), 0, s, p, (long)t->nparam, 0.f);
  PSWA_HIP_TRY(hipGetLastError());
  PSWA_HIP_TRY(hipStreamSynchronize(s));
  *out = t.release();
  return PSWA_OK;
}

pswa_status pswa_train_step(pswa_trainer* t, int B, int n_prev, const int32_t* d_latents,
                            const int32_t* d_hyper, const int32_t* d_prev, const float* d_mu_t,
                            const float* d_lsig_t, float lr, float weight_decay, int update,
                            double* h_loss, void* stream) {
  if (!t) return fail(PSWA_E_ARG, "trainer is null");
  if (B < 1 || B > t->Bmax) return fail(PSWA_E_ARG, "crop count %d outside [1, %d]", B, t->Bmax);
  if (n_prev != 0 && n_prev != 2) return fail(PSWA_E_ARG, "n_prev must be 0 or 2");
  if (!d_latents || !d_hyper || !d_mu_t || !d_lsig_t || (n_prev && !d_prev))
    return fail(PSWA_E_ARG, "null input pointer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const NetDims& x = t->x;
  const int d = x.d, F = x.F, C = x.C, dh = x.dh, L = x.L, hd = x.heads;
  const int HW = t->H * t->W;
  const long N = (long)B * HW, N2 = 2 * N;
  const bool P = n_prev != 0;
  float* w = t->w;
  float* g = t->g;
  auto Wp = [&](int k) { return T_(t, w, k); };
  auto Gp = [&](int k) { return T_(t, g, k); };
  const int nb_acc = x.n_acc, nb_lay = x.n_sp + x.n_tm;

  hipLaunchKernelGGL(k_fill, dim3(cdiv(t->nparam, kT)), dim3(kT), 0, s, g, (long)t->nparam, 0.f);

  // ------------------------------------------------------------ forward
  hipLaunchKernelGGL(k_to_float, dim3(cdiv(N * C, kT)), dim3(kT), 0, s, d_latents, Wp(I_ING),
                     t->yf, t->yg, N * C, C);
  if (P)
    hipLaunchKernelGGL(k_to_float, dim3(cdiv(N2 * C, kT)), dim3(kT), 0, s, d_prev, Wp(I_ING),
                       t->ypf, t->ypg, N2 * C, C);
  const long ncell = (long)B * t->Hh * t->Wh;
  hipLaunchKernelGGL(k_to_float, dim3(cdiv(ncell * x.Ch, kT)), dim3(kT), 0, s, d_hyper,
                     Wp(I_ING), t->zf, nullptr, ncell * x.Ch, x.Ch);
  for (int b = 0; b < B; ++b)
    hyper_embed(d_hyper + (size_t)b * t->Hh * t->Wh * x.Ch, t->Hh, t->Wh, x.Ch, Wp(I_HW),
                Wp(I_P4), t->H, t->W, d, t->h + (size_t)b * HW * d, s);
  lin(t, N, d, C, t->yg, C, Wp(I_INW), t->e, d, 0.f, s);
  if (P) lin(t, N2, d, C, t->ypg, C, Wp(I_INW), t->ep, d, 0.f, s);
  // accumulator
  rms_fwd(N, d, t->e, d, Wp(I_GKV), t->ukv, d, t->rkv, s);
  lin(t, N, 2 * d, d, t->ukv, d, Wp(I_WKV), t->KV0, 2 * d, 0.f, s);
  rms_fwd(N, d, t->h, d, Wp(I_GQ), t->uq, d, t->rq, s);
  lin(t, N, d, d, t->uq, d, Wp(I_WQ), t->Q0, d, 0.f, s);
  TAttn A0 = attn_args(t, N, true, false);
  A0.Q = t->Q0; A0.ldq = d;
  A0.K = t->KV0; A0.V = t->KV0 + d; A0.ldk = 2 * d;
  A0.knull = Wp(I_KNULL); A0.vnull = Wp(I_VNULL);
  A0.bias = Wp(I_ABIAS); A0.nbias = nb_acc;
  attn_fwd(A0, dh, t->A0, d, t->lse0, s);
  PSWA_HIP_TRY(hipMemcpyAsync(t->lay[0].x, t->h, N * d * sizeof(float), hipMemcpyDeviceToDevice, s));
  lin(t, N, d, d, t->A0, d, Wp(I_AWO), t->lay[0].x, d, 1.f, s);
  // layers
  std::vector<TAttn> La(L);
  for (int l = 0; l < L; ++l) {
    Lay& a = t->lay[l];
    rms_fwd(N, d, a.x, d, Wp(I_L(l, 0)), a.u, d, a.r1, s);
    lin(t, N, 3 * d, d, a.u, d, Wp(I_L(l, 1)), a.qkv, 3 * d, 0.f, s);
    if (P) {
      rms_fwd(N2, d, t->ep, d, Wp(I_L(l, 0)), a.up, d, a.rp, s);
      lin(t, N2, 2 * d, d, a.up, d, Wp(I_L(l, 1)) + (size_t)d * d, a.tkv, 2 * d, 0.f, s);
    }
    TAttn A = attn_args(t, N, false, P);
    A.Q = a.qkv; A.ldq = 3 * d;
    A.K = a.qkv + d; A.V = a.qkv + 2 * d; A.ldk = 3 * d;
    if (P) { A.Kt = a.tkv; A.Vt = a.tkv + d; A.ldt = 2 * d; }
    A.bias = Wp(I_L(l, 2)); A.nbias = nb_lay;
    attn_fwd(A, dh, a.att, d, a.lse, s);
    La[l] = A;
    PSWA_HIP_TRY(hipMemcpyAsync(a.y, a.x, N * d * sizeof(float), hipMemcpyDeviceToDevice, s));
    lin(t, N, d, d, a.att, d, Wp(I_L(l, 3)), a.y, d, 1.f, s);
    rms_fwd(N, d, a.y, d, Wp(I_L(l, 4)), a.v, d, a.r2, s);
    lin(t, N, F, d, a.v, d, Wp(I_L(l, 5)), a.g, F, 0.f, s);
    lin(t, N, F, d, a.v, d, Wp(I_L(l, 6)), a.upr, F, 0.f, s);
    hipLaunchKernelGGL(k_swiglu_fwd, dim3(cdiv(N * F, kT)), dim3(kT), 0, s, a.g, a.upr, a.hm, N * F);
    float* xo = t->lay[l + 1].x;
    PSWA_HIP_TRY(hipMemcpyAsync(xo, a.y, N * d * sizeof(float), hipMemcpyDeviceToDevice, s));
    lin(t, N, d, F, a.hm, F, Wp(I_L(l, 7)), xo, d, 1.f, s);
  }
  // head and loss
  const float* xL = t->lay[L].x;
  rms_fwd(N, d, xL, d, Wp(I_H(L, 0)), t->zh, d, t->rz, s);
  lin(t, N, d, d, t->zh, d, Wp(I_H(L, 1)), t->T1, d, 0.f, s);
  hipLaunchKernelGGL(k_silu_fwd, dim3(cdiv(N * d, kT)), dim3(kT), 0, s, t->T1, t->S1, N * d);
  lin(t, N, 2 * C, d, t->S1, d, Wp(I_H(L, 2)), t->T, 2 * C, 0.f, s);
  const long nsym = N * C;
  const int nlb = cdiv(nsym, kT);
  float* Pgm = t->Pg2;
  float* Pbm = t->Pg2 + nsym;
  float* Pgs = t->Pg2 + 2 * nsym;
  float* Pbs = t->Pg2 + 3 * nsym;
  hipLaunchKernelGGL(k_head_loss, dim3(nlb), dim3(kT), 0, s, t->T, int(N), C, Wp(I_H(L, 3)),
                     Wp(I_H(L, 4)), Wp(I_H(L, 5)), Wp(I_H(L, 6)), d_mu_t, d_lsig_t, x.ln_smin,
                     x.ln_smax, float(2.0 / double(nsym)), t->dT, Pgm, Pbm, Pgs, Pbs,
                     t->loss_part);
  PSWA_HIP_TRY(hipGetLastError());

  // ----------------------------------------------------------- backward
  colsum(t, Pgm, C, N, C, Gp(I_H(L, 3)), true, s);
  colsum(t, Pbm, C, N, C, Gp(I_H(L, 4)), true, s);
  colsum(t, Pgs, C, N, C, Gp(I_H(L, 5)), true, s);
  colsum(t, Pbs, C, N, C, Gp(I_H(L, 6)), true, s);
  lin_dx(t, N, 2 * C, d, t->dT, 2 * C, Wp(I_H(L, 2)), t->dS1, d, 0.f, s);
  lin_dw(t, N, 2 * C, d, t->dT, 2 * C, t->S1, d, Gp(I_H(L, 2)), s);
  hipLaunchKernelGGL(k_silu_bwd, dim3(cdiv(N * d, kT)), dim3(kT), 0, s, t->T1, t->dS1, t->dT1, N * d);
  lin_dx(t, N, d, d, t->dT1, d, Wp(I_H(L, 1)), t->dZ, d, 0.f, s);
  lin_dw(t, N, d, d, t->dT1, d, t->zh, d, Gp(I_H(L, 1)), s);
  rms_bwd(t, N, d, xL, d, Wp(I_H(L, 0)), t->rz, t->dZ, d, nullptr, 0, t->dX, d, Gp(I_H(L, 0)), s);
  if (P) hipLaunchKernelGGL(k_fill, dim3(cdiv(N2 * d, kT)), dim3(kT), 0, s, t->dEp, N2 * d, 0.f);

  for (int l = L - 1; l >= 0; --l) {
    Lay& a = t->lay[l];
    // MLP: x' = y + Wdown (silu(Wgate v) * Wup v), v = RMSNorm_g2(y)
    lin_dx(t, N, d, F, t->dX, d, Wp(I_L(l, 7)), t->dHm, F, 0.f, s);
    lin_dw(t, N, d, F, t->dX, d, a.hm, F, Gp(I_L(l, 7)), s);
    hipLaunchKernelGGL(k_swiglu_bwd, dim3(cdiv(N * F, kT)), dim3(kT), 0, s, a.g, a.upr, t->dHm,
                       t->dG, t->dUp, N * F);
    lin_dx(t, N, F, d, t->dG, F, Wp(I_L(l, 5)), t->dV, d, 0.f, s);
    lin_dx(t, N, F, d, t->dUp, F, Wp(I_L(l, 6)), t->dV, d, 1.f, s);
    lin_dw(t, N, F, d, t->dG, F, a.v, d, Gp(I_L(l, 5)), s);
    lin_dw(t, N, F, d, t->dUp, F, a.v, d, Gp(I_L(l, 6)), s);
    rms_bwd(t, N, d, a.y, d, Wp(I_L(l, 4)), a.r2, t->dV, d, t->dX, d, t->dY, d, Gp(I_L(l, 4)), s);
    // attention block: y = x + Wo att
    lin_dx(t, N, d, d, t->dY, d, Wp(I_L(l, 3)), t->dA, d, 0.f, s);
    lin_dw(t, N, d, d, t->dY, d, a.att, d, Gp(I_L(l, 3)), s);
    TAttn A = La[l];
    A.O = a.att;
    A.dO = t->dA;
    A.ldo = d;
    attn_bwd(t, A, dh, a.lse, t->dQKV, 3 * d, t->dQKV + d, t->dQKV + 2 * d, 3 * d, t->dTKV,
             t->dTKV + d, 2 * d, s);
    colsum(t, t->dSbuf, A.S * hd, N, A.S * hd, t->bias_tmp, false, s);
    hipLaunchKernelGGL(k_add_strided, dim3(cdiv(hd * A.S, kT)), dim3(kT), 0, s, t->bias_tmp, hd,
                       A.S, A.S, Gp(I_L(l, 2)), nb_lay);
    lin_dx(t, N, 3 * d, d, t->dQKV, 3 * d, Wp(I_L(l, 1)), t->dU, d, 0.f, s);
    lin_dw(t, N, 3 * d, d, t->dQKV, 3 * d, a.u, d, Gp(I_L(l, 1)), s);
    if (P) {
      lin_dw(t, N2, 2 * d, d, t->dTKV, 2 * d, a.up, d, Gp(I_L(l, 1)) + (size_t)d * d, s);
      lin_dx(t, N2, 2 * d, d, t->dTKV, 2 * d, Wp(I_L(l, 1)) + (size_t)d * d, t->dUP, d, 0.f, s);
      rms_bwd(t, N2, d, t->ep, d, Wp(I_L(l, 0)), a.rp, t->dUP, d, t->dEp, d, t->dEp, d,
              Gp(I_L(l, 0)), s);
    }
    rms_bwd(t, N, d, a.x, d, Wp(I_L(l, 0)), a.r1, t->dU, d, t->dY, d, t->dX, d, Gp(I_L(l, 0)), s);
  }

  // accumulator: x0 = h + Wo^a att
  lin_dx(t, N, d, d, t->dX, d, Wp(I_AWO), t->dA, d, 0.f, s);
  lin_dw(t, N, d, d, t->dX, d, t->A0, d, Gp(I_AWO), s);
  A0.O = t->A0;
  A0.dO = t->dA;
  A0.ldo = d;
  attn_bwd(t, A0, dh, t->lse0, t->dQ0, d, t->dKV0, t->dKV0 + d, 2 * d, nullptr, nullptr, 0, s);
  colsum(t, t->dSbuf, A0.S * hd, N, A0.S * hd, t->bias_tmp, false, s);
  hipLaunchKernelGGL(k_add_strided, dim3(cdiv(hd * nb_acc, kT)), dim3(kT), 0, s, t->bias_tmp, hd,
                     A0.S, nb_acc, Gp(I_ABIAS), nb_acc);
  {
    const int chunk = 256, nch = cdiv(N, chunk);
    hipLaunchKernelGGL(k_null_part, dim3(cdiv(2 * d, kT), nch), dim3(kT), 0, s, t->Pbuf,
                       t->dSbuf, A0.S, nb_acc, t->Q0, d, t->dA, d, int(N), d, dh, hd,
                       1.0f / std::sqrt(float(dh)), chunk, t->part);
    hipLaunchKernelGGL(k_colsum_final, dim3(cdiv(2 * d, kT)), dim3(kT), 0, s, t->part, nch,
                       2 * d, t->bias_tmp, 0);
    hipLaunchKernelGGL(k_add_strided, dim3(cdiv(d, kT)), dim3(kT), 0, s, t->bias_tmp, 1, d, d,
                       Gp(I_KNULL), d);
    hipLaunchKernelGGL(k_add_strided, dim3(cdiv(d, kT)), dim3(kT), 0, s, t->bias_tmp + d, 1, d, d,
                       Gp(I_VNULL), d);
  }
  lin_dx(t, N, d, d, t->dQ0, d, Wp(I_WQ), t->dU, d, 0.f, s);
  lin_dw(t, N, d, d, t->dQ0, d, t->uq, d, Gp(I_WQ), s);
  rms_bwd(t, N, d, t->h, d, Wp(I_GQ), t->rq, t->dU, d, t->dX, d, t->dH, d, Gp(I_GQ), s);
  lin_dx(t, N, 2 * d, d, t->dKV0, 2 * d, Wp(I_WKV), t->dU, d, 0.f, s);
  lin_dw(t, N, 2 * d, d, t->dKV0, 2 * d, t->ukv, d, Gp(I_WKV), s);
  rms_bwd(t, N, d, t->e, d, Wp(I_GKV), t->rkv, t->dU, d, nullptr, 0, t->dE, d, Gp(I_GKV), s);
  // latent embedding e = W_in (g_in * y) (and the previous frames' e)
  lin_dw(t, N, d, C, t->dE, d, t->yg, C, Gp(I_INW), s);
  lin_dx(t, N, d, C, t->dE, d, Wp(I_INW), t->dYg, C, 0.f, s);
  hipLaunchKernelGGL(k_mul, dim3(cdiv(N * C, kT)), dim3(kT), 0, s, t->dYg, t->yf, t->Pg, N * C);
  colsum(t, t->Pg, C, N, C, Gp(I_ING), true, s);
  if (P) {
    lin_dw(t, N2, d, C, t->dEp, d, t->ypg, C, Gp(I_INW), s);
    lin_dx(t, N2, d, C, t->dEp, d, Wp(I_INW), t->dYpg, C, 0.f, s);
    hipLaunchKernelGGL(k_mul, dim3(cdiv(N2 * C, kT)), dim3(kT), 0, s, t->dYpg, t->ypf, t->Pg,
                       N2 * C);
    colsum(t, t->Pg, C, N2, C, Gp(I_ING), true, s);
  }
  // hyperprior token h = W_h z_cell + P4[sub]
  hipLaunchKernelGGL(k_hyper_p4_grad, dim3(cdiv(16 * d, kT)), dim3(kT), 0, s, t->dH, B, t->H,
                     t->W, d, Gp(I_P4));
  hipLaunchKernelGGL(k_hyper_cell_sum, dim3(cdiv(ncell * d, kT)), dim3(kT), 0, s, t->dH, B, t->H,
                     t->W, t->Hh, t->Wh, d, t->dHc);
  lin_dw(t, ncell, d, x.Ch, t->dHc, d, t->zf, x.Ch, Gp(I_HW), s);
  PSWA_HIP_TRY(hipGetLastError());

  std::vector<float> lp(nlb);
  PSWA_HIP_TRY(hipMemcpyAsync(lp.data(), t->loss_part, nlb * sizeof(float), hipMemcpyDeviceToHost, s));
  if (update) {
    ++t->step;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = float(1.0 - std::pow(0.9, t->step)), c2 = float(1.0 - std::pow(0.999, t->step));
    for (size_t k = 0; k < t->span.size(); ++k) {
      const long n = (long)t->span[k].second;
      hipLaunchKernelGGL(k_adamw, dim3(cdiv(n, kT)), dim3(kT), 0, s, w + t->span[k].first,
                         g + t->span[k].first, t->m + t->span[k].first, t->v + t->span[k].first,
                         n, lr, decayed_tensor(int(k), L) ? weight_decay : 0.f, b1, b2, 1e-8f,
                         c1, c2);
    }
    PSWA_HIP_TRY(hipGetLastError());
  }
  PSWA_HIP_TRY(hipStreamSynchronize(s));
  if (h_loss) {
    double tot = 0;
    for (float v : lp) tot += v;
    *h_loss = tot / double(nsym);
  }
  return PSWA_OK;
}

pswa_status pswa_train_read(pswa_trainer* t, int what, float* h_blob, size_t blob_floats,
                            void* stream) {
  if (!t || !h_blob) return fail(PSWA_E_ARG, "null argument");
  if (what != 0 && what != 1) return fail(PSWA_E_ARG, "what must be 0 (weights) or 1 (gradients)");
  if (blob_floats != t->blob_floats)
    return fail(PSWA_E_SHAPE, "blob has %zu floats, model needs %zu", blob_floats, t->blob_floats);
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<float> padded(t->nparam);
  PSWA_HIP_TRY(hipMemcpyAsync(padded.data(), what == 0 ? t->w : t->g, t->nparam * sizeof(float),
                              hipMemcpyDeviceToHost, s));
  PSWA_HIP_TRY(hipStreamSynchronize(s));
  for (size_t k = 0; k < t->span.size(); ++k)
    std::memcpy(h_blob + t->span_blob[k].first, padded.data() + t->span[k].first,
                t->span[k].second * sizeof(float));
  return PSWA_OK;
}

int pswa_train_num_steps(const pswa_trainer* t) { return t ? t->step : -1; }

int pswa_student_accept(double bits_student, double bits_full, double max_overhead) {
  if (!(bits_student >= 0) || !(bits_full >= 0) || !(max_overhead >= 0)) return 0;
  return bits_student <= (1.0 + max_overhead) * bits_full ? 1 : 0;
}

void pswa_train_destroy(pswa_trainer* t) { delete t; }

}  // extern "C"
