/*
 * pswa.h -- C ABI of the MI355X (gfx950) P-SWA wavefront context model.
 *
 * Paper: Kopte and Kaup, "Parallel Context Modeling for Sliding Window
 * Attention in Neural Video Coding" (arXiv 2605.20977).
 *
 * The library predicts, for every symbol of a quantized latent y (H x W x C,
 * int32), the mean and scale of a Gaussian that drives an arithmetic coder
 * (Sec. 3.1 and Fig. 1: the prediction heads output mu and sigma), from
 *   - a hyperprior token per position (Sec. 3.1: the decoded hyperprior is
 *     the accumulator's query and residual),
 *   - an accumulator: cross-attention from that token to the already
 *     decoded neighbours (strictly past positions, Sec. 3.1 and Fig. 2b),
 *   - L causal sliding-window attention + SwiGLU layers (Sec. 3.1, Llama-2
 *     style blocks), joined for P-frames by a window over two previous frames,
 *   - a two-layer head with channel-wise output scales (Sec. 3.1).
 * Decoding walks a diagonal wavefront (Sec. 2, WPP; Sec. 3.2): position
 * (i, j) is decoded at step t = j + s*i with s = r + 1 for a k x k causal
 * window (r = (k-1)/2): the window holds all 2r+1 columns of the r rows above
 * and the r cells to the left, and every such cell lies on an earlier
 * diagonal. A frame takes T = (W-1) + s*(H-1) + 1 steps.
 *
 * Conventions shared by every call:
 *   - "d_" pointers are device pointers (HIP global memory), "h_" pointers
 *     are host pointers. Arrays are C-contiguous, raster order: a latent
 *     array [H][W][C] holds symbol (i, j, c) at (i*W + j)*C + c.
 *   - The caller owns all device memory (the model's weights region, the
 *     encode workspace, the decode state) and passes pointer + size; the
 *     library never calls hipMalloc/hipFree. Opaque handles are host objects
 *     owned by the library and freed by the matching *_destroy call.
 *   - `stream` is a hipStream_t (NULL = the null stream). All device work of
 *     a call is enqueued on it. A call returns before that work finishes
 *     unless it documents a wait.
 *   - Every call returns a pswa_status; no C++ exception crosses the ABI.
 *     pswa_last_error() returns the calling thread's last message. Argument
 *     and shape checks run before any HIP call.
 *   - Determinism: for one model and precision, pswa_encode_params and the
 *     pswa_decode_step sequence produce bit-identical mean, scale, bits,
 *     centre and table index (every kernel is shared and each row's
 *     reduction order does not depend on how many rows run together).
 */
#ifndef PSWA_H
#define PSWA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PSWA_OK = 0,
  PSWA_E_ARG = -1,         /* null pointer, bad enum, buffer too small   */
  PSWA_E_SHAPE = -2,       /* inconsistent sizes (e.g. Hh != ceil(H/4))  */
  PSWA_E_ORDER = -3,       /* decode_step called out of order            */
  PSWA_E_HIP = -4,         /* a HIP runtime call failed                  */
  PSWA_E_UNSUPPORTED = -5, /* valid request this build does not serve    */
  PSWA_E_CORRUPT = -6,     /* bitstream truncated or inconsistent        */
  PSWA_E_NUMERIC = -7      /* a non-finite mean/scale was produced       */
} pswa_status;

typedef enum { PSWA_FP32 = 0, PSWA_BF16 = 1, PSWA_FP8_E4M3 = 2 } pswa_precision;

enum { PSWA_SRC_DEVICE = 0, PSWA_SRC_BITSTREAM = 1 };

/* Model shape. window is odd (3..9); d a multiple of 64, <= 1024; head dim
 * d / heads in {16, 32, 48, 64}; mlp_ratio * d <= 2048; C a multiple of 4,
 * <= 256; Ch <= 512. Other shapes are rejected with PSWA_E_ARG. */
typedef struct {
  int32_t L, d, heads, window, mlp_ratio, C, Ch;
  int32_t prec;  /* pswa_precision */
  int32_t cycle; /* decoding schedule: 0 = wavefront t = j + s i with the causal
                    half-window (s = r + 1); c in [2, 16] = the cyclic pattern
                    step = (i + j) mod c over the full window, the accumulator
                    seeing strictly earlier steps and the layers steps up to
                    the query's own (Sec. 3.2, Fig. 2) */
  int32_t act_scaling; /* FP8 activation scaling (pswa_act_scaling); must be
                          PSWA_ACT_TENSOR for FP32 and BF16 models */
  /* Channel Transformer (Sec. 3.1; Sec. 3.2: N channel groups decoded one
   * after the other at every step). ch_groups = 0: the plain head (ch_d and
   * ch_L must be 0). ch_groups = N in [1, 8]: the latent's C channels are N
   * groups of C/N (a multiple of 4); the head is replaced by a channel
   * transformer of width ch_d (ch_d/N a multiple of 16 in [16, 512]) with
   * ch_L in [1, 4] blocks and a SwiGLU of ch_ratio (1..4) * ch_d/N per group,
   * and grouped two-layer heads. Its input is the spatial output (RMSNorm,
   * then a linear map) plus a linear map of the latent shifted by one group
   * (input scale first); each block adds a mixing map of the per-group
   * RMSNorm of its input, masked block-lower-triangular so that group g
   * reads groups 0..g only, then a per-group pre-norm SwiGLU. Group g's mean
   * and scale therefore depend on the symbols of groups < g of the same
   * position only. The channel transformer runs in FP32 in every precision;
   * models with channel groups serve pswa_encode_params, the device-source
   * decode and (FP32 models) the batched decode, where each step runs the
   * input map of every group, then group by group the latent map, the blocks
   * and the group's head (bitstream decoding, the batched decode of BF16 /
   * FP8 models and training return PSWA_E_UNSUPPORTED). */
  int32_t ch_groups, ch_d, ch_L, ch_ratio;
} pswa_model_desc;

/* How a PSWA_FP8_E4M3 model scales each projection input before rounding it
 * to FP8 (Sec. 4.2.2 runs the network in reduced precision; the per-tensor
 * form is the configured one):
 *   PSWA_ACT_TENSOR: one static scale per projection input, 448 / amax, from
 *     maxima calibrated offline (pswa_calibrate) and passed after the weight
 *     blob; values beyond amax saturate at +-448. For RMSNorm inputs the
 *     scaled value is the normalized row (times its gain).
 *   PSWA_ACT_ROW: each row scaled by 448 / its own maximum, computed in the
 *     tile (no calibration).
 * Either way every row's arithmetic depends on that row only, so encode,
 * decode and batch decode stay bit-identical. */
typedef enum { PSWA_ACT_TENSOR = 0, PSWA_ACT_ROW = 1 } pswa_act_scaling;

/* Frame shape. Hh = ceil(H/4), Wh = ceil(W/4) (the hyperprior is at a
 * quarter of the latent resolution, Fig. 1); n_prev = 0 (I-frame) or 2
 * (P-frame with the two previous latents). */
typedef struct {
  int32_t H, W, Hh, Wh, n_prev;
} pswa_frame_desc;

typedef struct pswa_model pswa_model;
typedef struct pswa_state pswa_state;

/* ---------------------------------------------------------------- model */

/* Number of float32 values in a weight blob for `desc`. The blob is the
 * concatenation, in this order, of (linear weights are [out][in]):
 *   hyper.W [d][Ch], hyper.P4 [16][d], in.g [C], in.W [d][C],
 *   acc.gq [d], acc.Wq [d][d], acc.gkv [d], acc.Wkv [2d][d], acc.knull [d],
 *   acc.vnull [d], acc.bias [heads][2r(r+1)], acc.Wo [d][d],
 *   per layer l = 0..L-1: g1 [d], Wqkv [3d][d], bias [heads][nS + nT],
 *     Wo [d][d], g2 [d], Wgate [F][d], Wup [F][d], Wdown [d][F],
 *   head.g [d], head.W1 [d][d], head.W2 [2C][d], head.gmu [C], head.bmu [C],
 *   head.gsig [C], head.bsig [C];
 * With channel groups (N = ch_groups, dc = ch_d, dg = dc/N, Cg = C/N,
 * Fg = ch_ratio*dg) head.g, head.W1 and head.W2 are replaced by
 *   ct.gx [d], ct.Wx [dc][d], ct.gy [C], ct.Wy [dc][C] (acting on the latent
 *   shifted by one group: its column block j holds latent group j-1, block 0
 *   zeros; only row group g's column blocks 0..g are used),
 *   per block b = 0..ch_L-1: ct<b>.g1 [dc], ct<b>.M [dc][dc] (only blocks
 *   (g, j) with j <= g are used), ct<b>.g2 [dc], ct<b>.Wgate [N][Fg][dg],
 *   ct<b>.Wup [N][Fg][dg], ct<b>.Wdown [N][dg][Fg],
 *   ctH.g [dc], ctH.W1 [N][dg][dg], ctH.W2 [N][2Cg][dg] (group g's means then
 *   scales);
 * with r = (window-1)/2, F = mlp_ratio*d, nS = 2r(r+1)+1 spatial bias slots
 * (the causal window in row-major order, then the query itself) and
 * nT = 2(2r+1)^2 temporal slots (previous frame 1 then 2, each its full
 * window in row-major order). For a PSWA_FP8_E4M3 model with
 * act_scaling = PSWA_ACT_TENSOR the weights are followed by
 * pswa_act_points(desc) floats: the calibrated absolute maximum of every
 * projection input (finite, >= 0; 0 gives the scale 1). Returns 0 for an
 * invalid desc. */
size_t pswa_model_blob_floats(const pswa_model_desc* desc);

/* Number of projection inputs, in this order: the latent embedding (in.W),
 * the accumulator's q, k/v and o projections, per layer the QKV, O, gate/up
 * (one input for both) and down projections, then head.W1 and head.W2:
 * 6 + 4 L. Returns 0 for an invalid desc. */
int pswa_act_points(const pswa_model_desc* desc);

/* Device bytes the model needs (weights plus their low-precision copies). */
size_t pswa_model_device_bytes(const pswa_model_desc* desc);

/* Upload a blob into caller-owned device memory d_mem (>= device_bytes,
 * 256-byte aligned). Waits for the upload (the blob may be freed on return).
 * For PSWA_BF16 / PSWA_FP8_E4M3 the projection and MLP weights are rounded
 * once (RNE; FP8 saturating, one static scale per tensor) and stored in the
 * matrix-core fragment order (private to the library; the FP32 weights stay
 * row-major); such models also keep every key/value cache (accumulator,
 * layers, temporal) in BF16, rounded to nearest even from the projection
 * output, with attention arithmetic in FP32 (state and workspace sizes are
 * those of FP32 caches). */
pswa_status pswa_model_create(const pswa_model_desc* desc, const float* h_blob,
                              size_t blob_floats, void* d_mem, size_t d_bytes,
                              void* stream, pswa_model** out);
void pswa_model_destroy(pswa_model* model);

/* ------------------------------------------------- encode (parallel form) */

size_t pswa_encode_workspace_bytes(const pswa_model* model,
                                   const pswa_frame_desc* frame);

/* Every position at once (the decoder's arithmetic, row for row).
 *   d_latents [H][W][C] int32, d_hyper [Hh][Wh][Ch] int32,
 *   d_prev [2][H][W][C] int32 (frame 1 = most recent) or NULL for I-frames;
 *   outputs [H][W][C]: d_mean, d_scale (float), d_bits (float, -log2 of the
 *   discretized-Gaussian mass, floored at 1e-9), d_cdf_center (int32) and
 *   d_cdf_index (uint16: table scale*16 + phase, see pswa_cdf_tables).
 *   h_total_bits: if non-NULL, waits and stores the sum of d_bits; the wait
 *   also reports PSWA_E_NUMERIC if any mean/scale was non-finite.
 *   d_ws: workspace of pswa_encode_workspace_bytes, 256-byte aligned. */
pswa_status pswa_encode_params(const pswa_model* model, const pswa_frame_desc* frame,
                               const int32_t* d_latents, const int32_t* d_hyper,
                               const int32_t* d_prev, float* d_mean, float* d_scale,
                               float* d_bits, int32_t* d_cdf_center,
                               uint16_t* d_cdf_index, double* h_total_bits,
                               void* d_ws, size_t ws_bytes, void* stream);

/* pswa_encode_params without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the workspace is the library's static
 * scratch array on the current device, pswa_noalloc_scratch_bytes() bytes
 * (64 MiB), held by every GPU the library runs on until the process ends.
 * Other arguments and outputs as in pswa_encode_params (the caller still
 * owns inputs and outputs). A frame whose workspace
 * (pswa_encode_workspace_bytes) exceeds the scratch is refused with
 * PSWA_E_UNSUPPORTED before any device work. Every call on one GPU shares
 * that GPU's scratch: calls that overlap on one GPU (other streams, other
 * threads) race, and must be serialized by the caller. The call clears what
 * must start at zero itself; the scratch keeps the last call's contents. */
size_t pswa_noalloc_scratch_bytes(void);
pswa_status pswa_encode_params_noalloc(const pswa_model* model, const pswa_frame_desc* frame,
                                       const int32_t* d_latents, const int32_t* d_hyper,
                                       const int32_t* d_prev, float* d_mean, float* d_scale,
                                       float* d_bits, int32_t* d_cdf_center,
                                       uint16_t* d_cdf_index, double* h_total_bits,
                                       void* stream);

/* Calibration of FP8 per-tensor activation scales: runs the encode form of
 * an FP32 model on one frame (arguments as in pswa_encode_params) and
 * max-combines into d_amax [pswa_act_points] (device float, zeroed by the
 * caller before the first frame) the largest |value| each projection
 * multiplies: the RMSNorm output (gain included) for normed inputs, the
 * latent times its input scale for the embedding, the raw input otherwise;
 * the temporal keys/values of P-frames count toward their layer's QKV input.
 * d_ws: pswa_calibrate_workspace_bytes, 256-byte aligned. Returns
 * PSWA_E_UNSUPPORTED for a model that is not FP32. Does not wait. */
size_t pswa_calibrate_workspace_bytes(const pswa_model* model, const pswa_frame_desc* frame);
pswa_status pswa_calibrate(const pswa_model* model, const pswa_frame_desc* frame,
                           const int32_t* d_latents, const int32_t* d_hyper,
                           const int32_t* d_prev, float* d_amax, void* d_ws, size_t ws_bytes,
                           void* stream);

/* ---------------------------------------------------------------- decode */

size_t pswa_state_bytes(const pswa_model* model, const pswa_frame_desc* frame);

/* Start decoding one frame: builds the hyperprior tokens and, for P-frames,
 * the per-layer keys/values of the two previous latents.
 *   symbol_source = PSWA_SRC_DEVICE: src is d_latents [H][W][C] int32 on the
 *     device; each step copies the symbols of its diagonal from there (the
 *     model-limited mode used for throughput and encode-by-decode checks).
 *   symbol_source = PSWA_SRC_BITSTREAM: src is a host byte array of
 *     src_bytes written by pswa_range_encode; each step waits for its CDF
 *     selections, range-decodes the diagonal on the CPU and uploads it.
 *   d_state_mem: pswa_state_bytes, 256-byte aligned, owned by the caller and
 *   untouched by anyone else until pswa_state_destroy. */
pswa_status pswa_decode_begin(const pswa_model* model, const pswa_frame_desc* frame,
                              const int32_t* d_hyper, const int32_t* d_prev,
                              int symbol_source, const void* src, size_t src_bytes,
                              void* d_state_mem, size_t state_bytes, void* stream,
                              pswa_state** out);

/* Number of wavefront steps T of the frame. */
int pswa_num_steps(const pswa_state* state);

/* Decode diagonal t = {(i, t - s*i)}: accumulator, L layers and head for
 * its positions, then the symbols (from the chosen source) and the
 * accumulator keys/values of the decoded positions. Steps must be called
 * for t = 0, 1, ..., T-1 in order, else PSWA_E_ORDER. */
pswa_status pswa_decode_step(pswa_state* state, int t, void* stream);

/* After the last step: copy out the decoded latents and (each optional,
 * NULL to skip) the per-symbol outputs, laid out as in pswa_encode_params.
 * h_total_bits waits as in pswa_encode_params. */
pswa_status pswa_decode_end(pswa_state* state, int32_t* d_latents_out, float* d_mean,
                            float* d_scale, float* d_bits, int32_t* d_cdf_center,
                            uint16_t* d_cdf_index, double* h_total_bits, void* stream);
void pswa_state_destroy(pswa_state* state);

/* ---------------------------------------------------- batched decode */

/* Persistent decode of many frames (any sizes, I and P mixed) in one launch:
 * one kernel walks the global steps t = 0 .. max_f T_f - 1, each step
 * holding the diagonal t of every frame that has one, with grid barriers
 * between the dependent phases of the network (Sec. 3.2: every position of
 * a diagonal is predicted in one step; the frames of a batch are
 * independent). Per-row arithmetic is the same as in pswa_decode_step and
 * pswa_encode_params, so the outputs are bit-identical to theirs. Symbols
 * come from device memory (one d_latents per frame). */
typedef struct {
  pswa_frame_desc frame;
  const int32_t* d_hyper;   /* [Hh][Wh][Ch] */
  const int32_t* d_prev;    /* [2][H][W][C] for P-frames, else NULL */
  const int32_t* d_latents; /* symbol source [H][W][C] */
} pswa_batch_frame;

typedef struct pswa_batch pswa_batch;

/* Workspace bytes for the batch (0 for invalid frames). The workspace holds
 * every frame's caches and outputs plus row and argument tables sized for
 * any grouping of the frames. */
size_t pswa_batch_workspace_bytes(const pswa_model* model, int n, const pswa_batch_frame* frames);

/* Plan a batch in caller-owned workspace (256-byte aligned): builds and
 * uploads the row and argument tables and waits for the upload. The frames
 * are split into groups, each decoded by its own persistent workgroups
 * behind its own barrier (frames never depend on each other). grid > 0: one
 * group of `grid` workgroups; grid = 0: a default grouping (8 to 32
 * workgroups per group). Grids are clamped to what can be co-resident. The
 * frames' device buffers must stay valid until pswa_batch_destroy. */
pswa_status pswa_batch_create(const pswa_model* model, int n, const pswa_batch_frame* frames,
                              int grid, void* d_ws, size_t ws_bytes, void* stream,
                              pswa_batch** out);

/* Enqueue one full decode of the batch: hyperprior tokens and previous-frame
 * keys of every frame, then the persistent launch. Does not wait; may be
 * called again to decode the same inputs again, and may be captured in a
 * HIP graph. */
pswa_status pswa_batch_run(pswa_batch* batch, void* stream);

/* Waits for the stream and reports a barrier-timeout abort (PSWA_E_HIP) or a
 * non-finite mean/scale (PSWA_E_NUMERIC) of the last run. */
pswa_status pswa_batch_check(pswa_batch* batch, void* stream);

/* Copy frame f's outputs (each optional) laid out as in pswa_encode_params;
 * h_total_bits waits (and checks, as pswa_batch_check). */
pswa_status pswa_batch_outputs(pswa_batch* batch, int f, int32_t* d_latents_out, float* d_mean,
                               float* d_scale, float* d_bits, int32_t* d_cdf_center,
                               uint16_t* d_cdf_index, double* h_total_bits, void* stream);

int pswa_batch_num_steps(const pswa_batch* batch);  /* global steps (longest frame) */
int pswa_batch_max_rows(const pswa_batch* batch);   /* rows of all frames at one step, max */
int pswa_batch_grid(const pswa_batch* batch);       /* workgroups of the launch */
int pswa_batch_max_grid(const pswa_batch* batch);   /* co-resident limit */
/* One group of `grid` workgroups for all frames; 1 <= grid <= max. Waits. */
pswa_status pswa_batch_set_grid(pswa_batch* batch, int grid);
/* Groups of at most frames_per_group frames with blocks_per_group
 * workgroups each (autotuner knobs); the number of groups times
 * blocks_per_group must not exceed the co-resident limit. Rebuilds and
 * uploads the tables on `stream` and waits. */
pswa_status pswa_batch_set_groups(pswa_batch* batch, int frames_per_group, int blocks_per_group,
                                  void* stream);
pswa_status pswa_batch_groups(const pswa_batch* batch, int* frames_per_group,
                              int* blocks_per_group, int* n_groups);
/* Rows per BF16/FP8 GEMM tile, 16 or 32 (an autotuner knob; it changes which
 * tile computes a row, never the row's arithmetic). FP32 models reject 16. */
pswa_status pswa_batch_set_rtile(pswa_batch* batch, int rtile);
int pswa_batch_rtile(const pswa_batch* batch);
/* Autotuner: times every grouping candidate (frames per group and blocks
 * per group in powers of two) with 32-row tiles, then 16-row tiles on the
 * best grouping (BF16/FP8), then the other attention form on the winner
 * (pswa_batch_set_attention; FP32 caches only), each on a window of the
 * widest global steps (reps timed runs, median), and keeps the fastest. With
 * cache_path, a result for the same device, model shape, schedule,
 * precision and frame mix is read from that file
 * (JSON lines) instead of timing, and new results are appended. Reports the
 * choice and the estimated whole-run time. Waits. */
pswa_status pswa_batch_autotune(pswa_batch* batch, const char* cache_path, int reps,
                                void* stream, int* out_frames_per_group,
                                int* out_blocks_per_group, int* out_rtile, float* out_ms);
/* Record one full run (as pswa_batch_run does it) into a HIP graph; later
 * pswa_batch_run calls launch the graph, which reads the frames' input
 * buffers as they are at launch time. While the kernel timer is on, runs are
 * issued kernel by kernel (same kernels, same arguments) so each is timed.
 * Changing the grouping, row tile, spin limit or trace buffer drops the
 * graph. The capture uses a private stream; the kernel timer must be off. */
pswa_status pswa_batch_capture(pswa_batch* batch, void* stream);
/* Barrier form (on by default): a group whose workgroups all run on one XCD
 * (checked by the kernel at every launch from the hardware XCD id) meets at
 * a barrier that keeps the XCD's shared L2 and only invalidates each CU's
 * L1; off, or for groups that span XCDs, every barrier is device-scope
 * (L2 written back and invalidated). Both give the same results. */
pswa_status pswa_batch_set_xcd_barrier(pswa_batch* batch, int on);
/* Attention form of the wavefront schedule (an autotuner knob; both give
 * the same bits): staged != 0 stages, per tile of up to four consecutive
 * diagonal rows of a frame, the union of their causal windows (K and V rows
 * of a few heads at a time, as the caches hold them: FP32, or BF16 for BF16
 * and FP8 models, the queries and the window biases) in LDS with direct
 * global-to-LDS loads and computes the rows' items from LDS; 0 lets every
 * lane load its key's rows from global memory. The cyclic schedule rejects
 * staged != 0 (PSWA_E_UNSUPPORTED). Drops a captured graph.
 * pswa_batch_attention returns the current form (-1 for a null batch). */
pswa_status pswa_batch_set_attention(pswa_batch* batch, int staged);
int pswa_batch_attention(const pswa_batch* batch);
/* Bound on the spin count of one barrier wait before the launch aborts
 * (default about a second of waiting). Lowering it forces the abort path. */
pswa_status pswa_batch_set_spin_limit(pswa_batch* batch, int64_t spins);
/* Phase timeline (a profiling aid): while d_trace is set, one thread of the
 * persistent kernel (rank 0 of group 0) writes the device wall clock
 * (100 MHz) when it reaches and when it leaves each of its group's barriers:
 * d_trace[2k] and d_trace[2k + 1] for barrier k, for 2k + 1 < n (device
 * int64). Barriers per step: 2 + 5 L + 4 (with channel groups N and
 * blocks B: 2 + 5 L + 2 + 1 + N (3 + 4 B) - 1). n = 0 turns the trace off. */
pswa_status pswa_batch_trace(pswa_batch* batch, int64_t* d_trace, int n);
void pswa_batch_destroy(pswa_batch* batch);

/* ------------------------------------------------ student distillation */

/* Training of a (student) context model to reproduce another model's mean
 * and log-scale: FP32, hand-written kernels, parallel form (teacher
 * forcing). Loss = mean over symbols of (mu - mu_t)^2 + (lsig - lsig_t)^2,
 * lsig the clamped log-scale (no gradient where the clamp is active);
 * AdamW with beta1 0.9, beta2 0.999, eps 1e-8 and decoupled weight decay on
 * the linear weights only. The trainer holds weights, gradients and moments
 * in caller-owned device memory; crops are frames of their own (borders
 * masked). */
typedef struct pswa_trainer pswa_trainer;

/* Workspace for batches of up to max_crops crops of H x W (0 if invalid;
 * the model must be FP32 with the wavefront schedule (cycle 0) and
 * max_crops * H * W <= 2^22). */
size_t pswa_train_workspace_bytes(const pswa_model_desc* student, int max_crops, int H, int W);
/* Initial weights from a host blob in the documented order (see
 * pswa_model_create). Waits for the upload. */
pswa_status pswa_train_create(const pswa_model_desc* student, const float* h_blob,
                              size_t blob_floats, int max_crops, int H, int W, void* d_ws,
                              size_t ws_bytes, void* stream, pswa_trainer** out);
/* One step on B crops (B <= max_crops): device int32 latents [B][H][W][C],
 * hyperpriors [B][ceil(H/4)][ceil(W/4)][Ch], previous latents
 * [B][2][H][W][C] when n_prev = 2 (else NULL), and the targets mu_t and
 * lsig_t [B][H][W][C] (float). Computes the loss and every gradient; with
 * update != 0 also applies one AdamW step (lr, weight_decay). h_loss gets
 * the loss. Waits. */
pswa_status pswa_train_step(pswa_trainer* trainer, int B, int n_prev, const int32_t* d_latents,
                            const int32_t* d_hyper, const int32_t* d_prev, const float* d_mu_t,
                            const float* d_lsig_t, float lr, float weight_decay, int update,
                            double* h_loss, void* stream);
/* Copy the current weights (what = 0) or the last step's gradients
 * (what = 1) into a host blob in the documented order. Waits. */
pswa_status pswa_train_read(pswa_trainer* trainer, int what, float* h_blob, size_t blob_floats,
                            void* stream);
int pswa_train_num_steps(const pswa_trainer* trainer);  /* AdamW steps taken */
void pswa_train_destroy(pswa_trainer* trainer);

/* Per-frame fallback: 1 when a frame coded with the student (bits_student,
 * from pswa_encode_params with the student model) stays within
 * max_overhead (a fraction, e.g. 0.01) of the full model's bits, else 0 (code
 * the frame with the full model; the choice is one flag in the stream). Any
 * negative or NaN argument gives 0. */
int pswa_student_accept(double bits_student, double bits_full, double max_overhead);

/* ---------------------------------------------------------- entropy side */

/* Table selection of n symbols from their mean and log-scale (float32
 * decision, one rounding per operation):
 *   centre c = floor(mu + 0.5); phase m = min(15, floor((mu - c + 0.5)*16));
 *   scale s = clamp(floor((ln_sigma - ln 0.11) * (63 / ln(64/0.11)) + 0.5), 0, 63);
 *   index = s*16 + m. */
pswa_status pswa_cdf_select(const float* d_mean, const float* d_log_scale, size_t n,
                            int32_t* d_center, uint16_t* d_index, void* stream);

/* The 1024 integer CDF tables (16-bit precision) on the host. Table
 * x = s*16 + m covers offsets -R..R from the centre plus an escape bin:
 * h_radius[x] = R, and its 2R+2 frequencies sit at h_freq[h_offset[x] ..].
 * Each frequency is max(1, floor(pmf * (65536 - n_bins))) of the float64
 * Gaussian mass with scale 0.11*exp(s*Delta), Delta = ln(64/0.11)/63, and
 * mean offset (m + 0.5)/16 - 0.5 (escape bin: both tails), and the rest of
 * 65536 goes to the largest bin (lowest index on ties).
 * h_offset holds 1025 entries; freq_cap is the capacity of h_freq in
 * entries (pass 0 with h_freq NULL to query the needed size in *h_offset[1024]). */
pswa_status pswa_cdf_tables(uint32_t* h_radius, uint32_t* h_offset, uint16_t* h_freq,
                            size_t freq_cap);

/* Range-code a frame's symbols in decode order (steps t = 0..T-1; within a
 * step rows i ascending for the wavefront, raster order for the cyclic
 * schedule; channels 0..C-1), each with its table: symbol v is coded as bin
 * v - c + R when |v - c| <= R, else as the escape bin followed by the sign
 * and an order-0 Exp-Golomb code of |v - c| - R - 1 in equiprobable bits.
 * All arrays are host [H][W][C]. window and cycle are the model's (they fix
 * the schedule). Writes at most cap bytes to out. */
pswa_status pswa_range_encode(const pswa_frame_desc* frame, int32_t C, int32_t window,
                              int32_t cycle, const int32_t* h_symbols, const int32_t* h_center,
                              const uint16_t* h_index, uint8_t* out, size_t cap,
                              size_t* out_bytes);

/* Decode n symbols coded with the given centres/indices (same coding as
 * above, in the given order); a host-only check of the coder. */
pswa_status pswa_range_decode_seq(const uint8_t* in, size_t in_bytes, size_t n,
                                  const int32_t* h_center, const uint16_t* h_index,
                                  int32_t* h_symbols_out);

/* Encode n symbols in the given order (the counterpart of the above). */
pswa_status pswa_range_encode_seq(size_t n, const int32_t* h_symbols,
                                  const int32_t* h_center, const uint16_t* h_index,
                                  uint8_t* out, size_t cap, size_t* out_bytes);

const char* pswa_last_error(void);

/* Host quantization used for projection weights (pswa_model_create):
 *   PSWA_BF16: h_out uint16 [n], bfloat16 of each value, round to nearest even;
 *   PSWA_FP8_E4M3: h_out uint8 [n], OCP FP8 e4m3fn (bias 7, max 448, no
 *     infinities) of value * s with the per-tensor scale s = 448 / max|value|
 *     (1 for an all-zero tensor), round to nearest even, saturating;
 *     *h_inv_scale = 1 / s.
 * PSWA_FP32 is rejected (nothing to do). */
pswa_status pswa_quantize(int prec, const float* h_in, size_t n, void* h_out, float* h_inv_scale);

/* ------------------------------------------------------------ profiling */

/* Live kernel timer (a profiling aid, off by default). While enabled, every
 * kernel the library launches is bracketed by two HIP events recorded on the
 * stream it is launched on, and its algorithmic bytes and flops (weights
 * once, activations in and out; 2 flops per multiply-add) are recorded under
 * the kernel's role. Enabling clears earlier records. Timing adds event
 * records between launches, so timed runs should not be the ones measured. */
pswa_status pswa_profile_enable(int on);

/* Number of roles (kernel kinds) the timer distinguishes. */
int pswa_profile_roles(void);

/* Totals of one role since the timer was enabled: waits for its events.
 * name (optional) receives the role's name. */
pswa_status pswa_profile_read(int role, char* name, size_t name_cap, double* total_ms,
                              int64_t* launches, double* alg_bytes, double* alg_flops);

#ifdef __cplusplus
}
#endif

#endif /* PSWA_H */
