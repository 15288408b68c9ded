// Batched persistent decode (C ABI in include/pswa.h): many frames of any
// sizes, I and P mixed, decoded in one persistent launch.
//
// All frames live in one global position space: frame f owns positions
// [off_f, off_f + H_f W_f). The frames are split into groups (frames per
// group and blocks per group are launch knobs); a group's rows at step t are
// the union of its frames' diagonal t. Frames never read each other's
// positions, so each group runs at its own pace behind its own barrier. The
// per-step row tables (global position and frame of each row) and argument
// tables are rebuilt on the host whenever the grouping changes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <memory>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/pswa.h"
#include "persistent.h"
#include "runtime.h"

using namespace pswa;

namespace {
// Blocks of a block map (device table), a bound on any grid.
constexpr int kMaxBlocks = 4096;
// Ints between two groups' barrier counters (separate 256-byte lines).
constexpr int kBarStride = 64;
}  // namespace

// One group of a grouping: its frames, steps, rows and table offsets.
struct GroupPlan {
  std::vector<int> frames;
  int T = 0, Mmax = 0;
  size_t row_off = 0;   // first activation row of the group
  size_t tab_off = 0;   // first step record of the group in the tables
  size_t pos_off = 0;   // first entry of the group in the row tables
  std::vector<int> row_start;  // [T + 1], relative to pos_off
};

struct pswa_batch {
  const pswa_model* model = nullptr;
  std::vector<pswa_batch_frame> frames;
  std::vector<FrameInfo> finfo;
  int HWt = 0, T = 0, Mmax = 0;
  int max_grid_r16 = 0, max_grid_r32 = 0;  // co-resident blocks per row tile
  int max_grid() const { return rtile == 16 ? max_grid_r16 : max_grid_r32; }
  int fpg = 1, bpg = 1, grid = 0;       // frames and blocks per group, total blocks
  std::vector<GroupPlan> groups;
  size_t rows_cap = 0, steps_cap = 0;   // worst case over groupings
  long spin_limit = 1L << 21;  // barrier wait bound (about a second)
  double alg_bytes = 0, alg_flops = 0;  // one persistent launch, for the timer
  long long* trace = nullptr;
  int trace_len = 0;
  int rtile = 32;                       // A rows per MFMA tile (16 or 32)
  int attn_staged = 0;                  // attention form (wavefront schedule)
  hipGraphExec_t graph = nullptr;       // captured run (pswa_batch_capture)
  ~pswa_batch() {
    if (graph) (void)hipGraphExecDestroy(graph);
  }
  bool any_p = false;
  // device (inside the caller's workspace)
  FrameInfo* d_frames = nullptr;
  int *gpos_all = nullptr, *fid_all = nullptr;
  float *h = nullptr, *acc_kv = nullptr, *kv = nullptr, *tkv = nullptr, *e_prev = nullptr;
  float* q_acc = nullptr;  // accumulator queries of every position, before the launch
  int32_t *ysrc = nullptr, *ydec = nullptr;
  float *mean = nullptr, *scale = nullptr, *bits = nullptr;
  int32_t* center = nullptr;
  uint16_t* index = nullptr;
  Acts a{};
  int* ctl = nullptr;   // [1] abort, [2] numeric flag
  int* bars = nullptr;  // [frames][kBarStride]: group barrier counters
  GroupInfo* d_groups = nullptr;
  int* block_map = nullptr;
  int* xcd_tab = nullptr;
  int xcd_local = 1;
  GemmArgs* gtab = nullptr;  // per-group, per-step argument tables
  AttnArgs* atab = nullptr;
  SymArgs* stab = nullptr;
  float* sum = nullptr;
  size_t bytes = 0;
};

namespace {

// LDS-staged window tiles serve the wavefront schedule (FP32 or BF16
// key/value caches).
bool staged_ok(const pswa_model* m) { return !m->x.cycle; }

// Frame layout of a batch and the worst-case sizes of any grouping: rows of
// all groups together (at most the sum of each frame's longest diagonal)
// and step records (at most the sum of each frame's steps).
struct Plan {
  std::vector<FrameInfo> finfo;
  int HWt = 0, T = 0, Mmax = 0;
  size_t rows_cap = 0, steps_cap = 0;
  bool any_p = false;
};

Plan make_plan(const NetDims& x, int n, const pswa_batch_frame* fr) {
  Plan p;
  int off = 0;
  for (int f = 0; f < n; ++f) {
    const pswa_frame_desc& d = fr[f].frame;
    p.finfo.push_back(FrameInfo{d.H, d.W, off, d.n_prev});
    off += d.H * d.W;
    const int T = sched_steps(x, d.H, d.W);
    p.T = std::max(p.T, T);
    p.steps_cap += T;
    int mf = 0;
    for (int t = 0; t < T; ++t) mf = std::max(mf, sched_len(x, d.H, d.W, t));
    p.rows_cap += mf;
    p.any_p = p.any_p || d.n_prev > 0;
  }
  p.HWt = off;
  for (int t = 0; t < p.T; ++t) {
    int cnt = 0;
    for (int f = 0; f < n; ++f) cnt += sched_len(x, fr[f].frame.H, fr[f].frame.W, t);
    p.Mmax = std::max(p.Mmax, cnt);
  }
  return p;
}

void lay_out(const NetDims& x, const Plan& p, int n, void* base, pswa_batch* b) {
  Layout L(base);
  const size_t HWt = p.HWt;
  b->d_frames = L.take<FrameInfo>(n);
  b->gpos_all = L.take<int>(HWt);
  b->fid_all = L.take<int>(HWt);
  b->h = L.take<float>(HWt * x.d);
  b->q_acc = L.take<float>(HWt * x.d);
  b->acc_kv = L.take<float>((HWt + 1) * 2 * x.d);  // + the null row
  b->kv = L.take<float>((size_t)x.L * HWt * 2 * x.d);
  b->tkv = p.any_p ? L.take<float>((size_t)x.L * 2 * HWt * 2 * x.d) : nullptr;
  b->e_prev = p.any_p ? L.take<float>(2 * HWt * x.d) : nullptr;
  b->ysrc = L.take<int32_t>(HWt * x.C);
  b->ydec = L.take<int32_t>(HWt * x.C);
  b->mean = L.take<float>(HWt * x.C);
  b->scale = L.take<float>(HWt * x.C);
  b->bits = L.take<float>(HWt * x.C);
  b->center = L.take<int32_t>(HWt * x.C);
  b->index = L.take<uint16_t>(HWt * x.C);
  b->a = take_acts(L, x, std::max<size_t>(p.rows_cap, 1));
  b->ctl = L.take<int>(64);
  b->bars = L.take<int>((size_t)n * kBarStride);
  b->d_groups = L.take<GroupInfo>(n);
  b->block_map = L.take<int>(kMaxBlocks);
  b->xcd_tab = L.take<int>(kMaxBlocks);
  b->sum = L.take<float>(64);
  b->gtab = L.take<GemmArgs>(p.steps_cap * gemm_phases(x.L, ct_phases(x)));
  b->atab = L.take<AttnArgs>(p.steps_cap * attn_phases(x.L));
  b->stab = L.take<SymArgs>(p.steps_cap);
  b->bytes = L.used;
}

pswa_status check_frames(const pswa_model* m, int n, const pswa_batch_frame* fr) {
  if (!m) return fail(PSWA_E_ARG, "model is null");
  if (m->x.cg && m->w.prec != PSWA_PREC_F32)
    return fail(PSWA_E_UNSUPPORTED,
                "the persistent decode of models with channel groups runs FP32 models only");
  if (n < 1 || !fr) return fail(PSWA_E_ARG, "need at least one frame");
  for (int f = 0; f < n; ++f) {
    std::string why;
    if (!valid_frame(&fr[f].frame, &why))
      return fail(PSWA_E_SHAPE, "frame %d: %s", f, why.c_str());
    if (!fr[f].d_hyper || !fr[f].d_latents) return fail(PSWA_E_ARG, "frame %d: null pointer", f);
    if ((fr[f].frame.n_prev != 0) != (fr[f].d_prev != nullptr))
      return fail(PSWA_E_ARG, "frame %d: d_prev must be given exactly for P-frames", f);
  }
  int64_t tot = 0;
  for (int f = 0; f < n; ++f) tot += (int64_t)fr[f].frame.H * fr[f].frame.W;
  if (tot > (1 << 24)) return fail(PSWA_E_SHAPE, "batch holds more than 2^24 positions");
  return PSWA_OK;
}

// Buffers of the batch as a pass context for one group (M, gpos and fid
// are set per step); the group's activations start at its first row.
PassCtx batch_ctx(const pswa_batch* b, const GroupPlan& g) {
  const NetDims& x = b->model->x;
  PassCtx c{};
  c.frames = b->d_frames;
  c.frame0 = b->finfo[g.frames[0]];
  c.HWt = b->HWt;
  c.h = b->h;
  c.acc_kv = b->acc_kv;
  c.kv = b->kv;
  c.kv_stride = (size_t)b->HWt * 2 * x.d;
  c.tkv = b->any_p ? b->tkv : nullptr;
  c.tkv_stride = (size_t)2 * b->HWt * 2 * x.d;
  const size_t r = g.row_off;
  c.x = b->a.x + r * x.d;
  c.q = b->a.q + r * x.d;
  c.att = b->a.att + r * x.d;
  c.e = b->a.e + r * x.d;
  c.t1 = b->a.t1 + r * x.d;
  c.hmid = b->a.hmid + r * x.F;
  if (x.cg) {
    c.ct_c = b->a.ct_c + r * x.cd;
    c.ct_u = b->a.ct_u + r * x.cd;
    c.ct_u_stride = b->rows_cap * x.cd;  // blocks of [rows_cap][cd]
    c.ct_h = b->a.ct_h + r * x.cFg;
    c.ct_t1 = b->a.ct_t1 + r * x.cdg;
  }
  c.mean = b->mean; c.scale = b->scale; c.bits = b->bits;
  c.center = b->center; c.index = b->index;
  c.center_c = nullptr; c.index_c = nullptr;
  c.flag = b->ctl + 2;
  c.ysrc = b->ysrc;
  c.src_compact = 0;
  c.ydec = b->ydec;
  return c;
}

// Argument tables of one group's steps and phases, in the kernel's order.
void build_tables(const pswa_batch* b, const GroupPlan& g, std::vector<GemmArgs>* gt,
                  std::vector<AttnArgs>* at, std::vector<SymArgs>* stb) {
  const NetDims& x = b->model->x;
  const DevWeights& w = b->model->w;
  const PassCtx base = batch_ctx(b, g);
  for (int t = 0; t < g.T; ++t) {
    PassCtx c = base;
    c.M = g.row_start[t + 1] - g.row_start[t];
    c.gpos = b->gpos_all + g.pos_off + g.row_start[t];
    c.fid = b->fid_all + g.pos_off + g.row_start[t];
    gt->push_back(args_acc_q(x, w, c));  // (computed before the launch, kept for the layout)
    gt->push_back(args_acc_o(x, w, c));
    AttnArgs aa = args_acc_attn(x, w, c);  // queries of the rows' positions
    aa.q = b->q_acc;
    aa.qrow = c.gpos;
    aa.ldq = x.d;
    at->push_back(aa);
    for (int l = 0; l < x.L; ++l) {
      gt->push_back(args_qkv(x, w, c, l));
      gt->push_back(args_o(x, w, c, l));
      gt->push_back(args_gateup(x, w, c, l));
      gt->push_back(args_down(x, w, c, l));
      at->push_back(args_attn(x, w, c, l));
    }
    gt->push_back(args_head1(x, w, c));
    // the persistent kernel gathers the step's symbols and computes their bits
    // in the head epilogue (no separate symbols phase)
    GemmArgs h2 = args_head2(x, w, c);
    h2.head.ysrc = c.ysrc;
    h2.head.src_compact = c.src_compact;
    h2.head.ydec = c.ydec;
    h2.head.bits = c.bits;
    gt->push_back(h2);
    gt->push_back(args_embed(x, w, c));
    gt->push_back(args_acc_kv(x, w, c));
    if (x.cg) {  // the Channel Transformer's entries (the head entries above go unused)
      GemmArgs in = args_ct_in(x, w, c, 0);  // every group's input map at once
      in.N = x.cd;
      gt->push_back(in);
      for (int g = 0; g < x.cg; ++g) {
        gt->push_back(g > 0 ? args_ct_latent(x, w, c, g) : gemm_base(0, x.cdg, x.cCg, R_HEAD1));
        for (int bl = 0; bl < x.cL; ++bl) {
          gt->push_back(args_ct_rms(x, w, c, bl, g));
          gt->push_back(args_ct_mix(x, w, c, bl, g));
          gt->push_back(args_ct_gateup(x, w, c, bl, g));
          gt->push_back(args_ct_down(x, w, c, bl, g));
        }
        gt->push_back(args_ct_head1(x, w, c, g));
        GemmArgs ch2 = args_ct_head2(x, w, c, g);  // also gathers the group's symbols
        ch2.head.ysrc = c.ysrc;
        ch2.head.src_compact = c.src_compact;
        ch2.head.ydec = c.ydec;
        ch2.head.bits = c.bits;
        gt->push_back(ch2);
      }
    }
    stb->push_back(SymArgs{c.M, x.C, c.gpos, c.ysrc, c.src_compact, c.ydec, c.mean, c.scale,
                           c.bits});
  }
}

PersistArgs persist_args(const pswa_batch* b) {
  PersistArgs P{};
  P.groups = b->d_groups;
  P.block_map = b->block_map;
  P.L = b->model->x.L;
  P.t_begin = 0;
  P.t_end = b->T;
  P.abort_flag = b->ctl + 1;
  P.spin_limit = b->spin_limit;
  P.trace = b->trace;
  P.trace_len = b->trace_len;
  P.xcd_tab = b->xcd_tab;
  P.xcd_local = b->xcd_local;
  P.cycle = b->model->x.cycle;
  P.ct_groups = b->model->x.cg;
  P.ct_blocks = b->model->x.cL;
  P.attn_staged = b->attn_staged && staged_ok(b->model);
  return P;
}

// Any change to the launch configuration invalidates a captured graph.
void drop_graph(pswa_batch* b) {
  if (b->graph) {
    (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
  }
}

void count_work(pswa_batch* b, const std::vector<GemmArgs>& gt,
                const std::vector<AttnArgs>& at, const std::vector<SymArgs>& stb);

// Split the frames into groups of at most fpg frames (frames with the most
// steps spread first, so groups get similar work), give each group bpg
// blocks, and rebuild and upload every row and argument table. Blocks are
// numbered across the XCDs in dispatch order (block b runs on XCD b mod 8),
// so a group's blocks sit on as few XCDs as possible. Waits for the upload.
pswa_status apply_groups(pswa_batch* b, int fpg, int bpg, hipStream_t st) {
  const NetDims& x = b->model->x;
  const int n = (int)b->finfo.size();
  if (fpg < 1 || bpg < 1) return fail(PSWA_E_ARG, "frames and blocks per group must be >= 1");
  fpg = std::min(fpg, n);
  const int ng = (n + fpg - 1) / fpg;
  if ((long)ng * bpg > b->max_grid() || (long)ng * bpg > kMaxBlocks)
    return fail(PSWA_E_ARG, "%d groups of %d blocks exceed the co-resident limit %d", ng, bpg,
                b->max_grid());
  std::vector<int> order(n);
  for (int f = 0; f < n; ++f) order[f] = f;
  std::stable_sort(order.begin(), order.end(), [&](int u, int v) {
    return b->finfo[u].H * b->finfo[u].W > b->finfo[v].H * b->finfo[v].W;
  });
  std::vector<GroupPlan> groups(ng);
  for (int k = 0; k < n; ++k) groups[k % ng].frames.push_back(order[k]);
  std::vector<int> gpos, fid;
  size_t row_off = 0, tab_off = 0;
  for (GroupPlan& g : groups) {
    std::sort(g.frames.begin(), g.frames.end());
    for (int f : g.frames) g.T = std::max(g.T, sched_steps(x, b->finfo[f].H, b->finfo[f].W));
    g.row_off = row_off;
    g.tab_off = tab_off;
    g.pos_off = gpos.size();
    g.row_start.assign(g.T + 1, 0);
    for (int t = 0; t < g.T; ++t) {
      int cnt = 0;
      for (int f : g.frames) {
        const FrameInfo& fi = b->finfo[f];
        sched_for_each(x, fi.H, fi.W, t, [&](int i, int j) {
          gpos.push_back(fi.off + i * fi.W + j);
          fid.push_back(f);
          ++cnt;
        });
      }
      g.row_start[t + 1] = g.row_start[t] + cnt;
      g.Mmax = std::max(g.Mmax, cnt);
    }
    row_off += g.Mmax;
    tab_off += g.T;
  }
  if (row_off > b->rows_cap || tab_off > b->steps_cap || gpos.size() != (size_t)b->HWt)
    return fail(PSWA_E_ARG, "internal: grouping exceeds its workspace");
  std::vector<GemmArgs> gt;
  std::vector<AttnArgs> at;
  std::vector<SymArgs> stb;
  std::vector<GroupInfo> gi(ng);
  const int na = attn_phases(x.L), ngm = gemm_phases(x.L, ct_phases(x));
  for (int k = 0; k < ng; ++k) {
    const GroupPlan& g = groups[k];
    build_tables(b, g, &gt, &at, &stb);
    gi[k].gtab = b->gtab + g.tab_off * ngm;
    gi[k].atab = b->atab + g.tab_off * na;
    gi[k].stab = b->stab + g.tab_off;
    gi[k].T = g.T;
    gi[k].nblocks = bpg;
    gi[k].bar = reinterpret_cast<unsigned*>(b->bars + (size_t)k * kBarStride);
  }
  const int grid = ng * bpg;
  std::vector<int> bmap(grid), xcd_order;
  for (int xc = 0; xc < 8; ++xc)
    for (int blk = xc; blk < grid; blk += 8) xcd_order.push_back(blk);
  for (int p = 0; p < grid; ++p) bmap[xcd_order[p]] = ((p / bpg) << 16) | (p % bpg);
  PSWA_HIP_TRY(hipMemcpyAsync(b->gpos_all, gpos.data(), gpos.size() * sizeof(int),
                              hipMemcpyHostToDevice, st));
  PSWA_HIP_TRY(hipMemcpyAsync(b->fid_all, fid.data(), fid.size() * sizeof(int),
                              hipMemcpyHostToDevice, st));
  PSWA_HIP_TRY(hipMemcpyAsync(b->gtab, gt.data(), gt.size() * sizeof(GemmArgs),
                              hipMemcpyHostToDevice, st));
  PSWA_HIP_TRY(hipMemcpyAsync(b->atab, at.data(), at.size() * sizeof(AttnArgs),
                              hipMemcpyHostToDevice, st));
  PSWA_HIP_TRY(hipMemcpyAsync(b->stab, stb.data(), stb.size() * sizeof(SymArgs),
                              hipMemcpyHostToDevice, st));
  PSWA_HIP_TRY(hipMemcpyAsync(b->d_groups, gi.data(), gi.size() * sizeof(GroupInfo),
                              hipMemcpyHostToDevice, st));
  PSWA_HIP_TRY(hipMemcpyAsync(b->block_map, bmap.data(), bmap.size() * sizeof(int),
                              hipMemcpyHostToDevice, st));
  PSWA_HIP_TRY(hipStreamSynchronize(st));
  b->groups = std::move(groups);
  b->fpg = fpg;
  b->bpg = bpg;
  b->grid = grid;
  count_work(b, gt, at, stb);
  drop_graph(b);
  return PSWA_OK;
}

pswa_status run(pswa_batch* b, hipStream_t st) {
  if (b->graph && !prof_on()) {
    PSWA_HIP_TRY(hipGraphLaunch(b->graph, st));
    return PSWA_OK;
  }
  const pswa_model* m = b->model;
  const NetDims& x = m->x;
  zero_ints(b->ctl, 3, st);
  zero_ints(b->bars, (int)b->groups.size() * kBarStride, st);
  null_row(b->acc_kv, b->HWt, m->w.knull, m->w.vnull, x.d, m->w.kv16, st);
  for (size_t f = 0; f < b->frames.size(); ++f) {
    const pswa_batch_frame& fr = b->frames[f];
    const FrameInfo& fi = b->finfo[f];
    const int HW = fi.H * fi.W;
    hyper_embed(fr.d_hyper, fr.frame.Hh, fr.frame.Wh, x.Ch, m->w.hyperW, m->w.P4, fi.H, fi.W,
                x.d, b->h + (size_t)fi.off * x.d, st);
    PSWA_HIP_TRY(hipMemcpyAsync(b->ysrc + (size_t)fi.off * x.C, fr.d_latents,
                                (size_t)HW * x.C * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    if (fi.n_prev) {
      embed_prev(m, HW, b->HWt, fi.off, fr.d_prev, b->e_prev, st);
      for (int l = 0; l < x.L; ++l)
        temporal_kv_layer(m, HW, b->HWt, fi.off, b->e_prev, l,
                          b->tkv + (size_t)l * 2 * b->HWt * 2 * x.d, st);
    }
  }
  {  // the accumulator's queries depend on the hyperprior tokens only
    PassCtx c{};
    c.M = b->HWt;
    c.h = b->h;
    c.q = b->q_acc;
    gemm_run(A_FLOAT, true, EPI_STORE, args_acc_q(x, m->w, c), st);
  }
  const int ev = prof_begin(st);
  launch_persistent(persist_args(b), m->x, m->w.prec, b->rtile, b->grid, st);
  prof_end(ev, st, R_PERSIST, b->alg_bytes, b->alg_flops);
  PSWA_HIP_TRY(hipGetLastError());
  return PSWA_OK;
}

// Algorithmic bytes and flops of one persistent launch: the per-phase
// figures of the per-launch path (weights once per phase, activations in and
// out, every window slot's K and V rows) summed over every step.
void count_work(pswa_batch* b, const std::vector<GemmArgs>& gt,
                const std::vector<AttnArgs>& at, const std::vector<SymArgs>& stb) {
  const NetDims& x = b->model->x;
  // (the spatial network's entries; Channel Transformer entries are not counted)
  const int ng = gemm_phases(x.L), ngs = gemm_phases(x.L, ct_phases(x)), na = attn_phases(x.L);
  static const Epi epis_head[4] = {EPI_SILU, EPI_HEAD, EPI_STORE, EPI_STORE};
  double by = 0, fl = 0;
  for (size_t t = 0; t < stb.size(); ++t) {
    if (stb[t].M == 0) continue;
    for (int k = 0; k < ng; ++k) {
      const GemmArgs& a = gt[(size_t)t * ngs + k];
      Epi e;
      if (k == 0) e = EPI_STORE;
      else if (k == 1) e = EPI_RESID;
      else if (k < 2 + 4 * x.L) {
        const int r = (k - 2) % 4;
        e = r == 0 ? EPI_QKV : r == 2 ? EPI_SWIGLU : EPI_RESID;
      } else {
        e = epis_head[k - 2 - 4 * x.L];
      }
      by += gemm_alg_bytes(a, e);
      fl += 2.0 * a.M * a.N * a.K * ((e == EPI_SWIGLU || e == EPI_HEAD) ? 2.0 : 1.0);
    }
    for (int k = 0; k < na; ++k) {
      const AttnArgs& a = at[(size_t)t * na + k];
      by += attn_alg_bytes(a);
      const double keys = attn_slots(a);
      fl += double(a.M) * a.heads * keys * 4.0 * a.dh;
    }
    by += 16.0 * stb[t].M * x.C + 4.0 * stb[t].M;  // symbols and bits
  }
  b->alg_bytes = by;
  b->alg_flops = fl;
}

}  // namespace

extern "C" {

size_t pswa_batch_workspace_bytes(const pswa_model* model, int n, const pswa_batch_frame* frames) {
  if (check_frames(model, n, frames) != PSWA_OK) return 0;
  Plan p = make_plan(model->x, n, frames);
  pswa_batch tmp;
  lay_out(model->x, p, n, nullptr, &tmp);
  return tmp.bytes;
}

pswa_status pswa_batch_create(const pswa_model* model, int n, const pswa_batch_frame* frames,
                              int grid, void* d_ws, size_t ws_bytes, void* stream,
                              pswa_batch** out) {
  if (!out) return fail(PSWA_E_ARG, "out is null");
  *out = nullptr;
  const pswa_status cs = check_frames(model, n, frames);
  if (cs != PSWA_OK) return cs;
  if (!d_ws || (reinterpret_cast<uintptr_t>(d_ws) % kAlign) != 0)
    return fail(PSWA_E_ARG, "workspace must be non-null and 256-byte aligned");
  Plan p = make_plan(model->x, n, frames);
  std::unique_ptr<pswa_batch> b(new pswa_batch);
  lay_out(model->x, p, n, d_ws, b.get());
  if (ws_bytes < b->bytes) return fail(PSWA_E_ARG, "workspace %zu bytes < %zu", ws_bytes, b->bytes);
  b->model = model;
  b->frames.assign(frames, frames + n);
  b->finfo = p.finfo;
  b->HWt = p.HWt;
  b->T = p.T;
  b->Mmax = p.Mmax;
  b->rows_cap = p.rows_cap;
  b->steps_cap = p.steps_cap;
  b->any_p = p.any_p;
  b->max_grid_r32 = std::min(persistent_max_grid(model->x, model->w.prec, 32), kMaxBlocks);
  b->max_grid_r16 = model->w.prec == PSWA_PREC_F32
                        ? b->max_grid_r32
                        : std::min(persistent_max_grid(model->x, model->w.prec, 16), kMaxBlocks);
  if (b->max_grid_r32 <= 0 || b->max_grid_r16 <= 0)
    return fail(PSWA_E_HIP, "cannot size the persistent grid");
  hipStream_t st = static_cast<hipStream_t>(stream);
  PSWA_HIP_TRY(hipMemcpyAsync(b->d_frames, p.finfo.data(), n * sizeof(FrameInfo),
                              hipMemcpyHostToDevice, st));
  int fpg, bpg;
  if (grid > 0) {  // one group of `grid` blocks
    fpg = n;
    bpg = std::min(grid, b->max_grid());
  } else {         // about 8 to 32 blocks per group, as many groups as fit
    bpg = 8;
    while (bpg < 32 && (long)n * bpg * 2 <= b->max_grid()) bpg *= 2;
    const int ng = std::max(1, std::min(n, b->max_grid() / bpg));
    fpg = (n + ng - 1) / ng;
  }
  const pswa_status gs = apply_groups(b.get(), fpg, bpg, st);
  if (gs != PSWA_OK) return gs;
  *out = b.release();
  return PSWA_OK;
}

int pswa_batch_num_steps(const pswa_batch* b) { return b ? b->T : -1; }
int pswa_batch_max_rows(const pswa_batch* b) { return b ? b->Mmax : -1; }
int pswa_batch_grid(const pswa_batch* b) { return b ? b->grid : -1; }
int pswa_batch_max_grid(const pswa_batch* b) { return b ? b->max_grid() : -1; }

pswa_status pswa_batch_set_grid(pswa_batch* b, int grid) {
  if (!b) return fail(PSWA_E_ARG, "batch is null");
  if (grid < 1 || grid > b->max_grid())
    return fail(PSWA_E_ARG, "grid %d outside [1, %d]", grid, b->max_grid());
  return apply_groups(b, (int)b->finfo.size(), grid, nullptr);
}

pswa_status pswa_batch_set_groups(pswa_batch* b, int frames_per_group, int blocks_per_group,
                                  void* stream) {
  if (!b) return fail(PSWA_E_ARG, "batch is null");
  return apply_groups(b, frames_per_group, blocks_per_group, static_cast<hipStream_t>(stream));
}

pswa_status pswa_batch_groups(const pswa_batch* b, int* frames_per_group, int* blocks_per_group,
                              int* n_groups) {
  if (!b) return fail(PSWA_E_ARG, "batch is null");
  if (frames_per_group) *frames_per_group = b->fpg;
  if (blocks_per_group) *blocks_per_group = b->bpg;
  if (n_groups) *n_groups = (int)b->groups.size();
  return PSWA_OK;
}

pswa_status pswa_batch_set_rtile(pswa_batch* b, int rtile) {
  if (!b) return fail(PSWA_E_ARG, "batch is null");
  if (rtile != 16 && rtile != 32) return fail(PSWA_E_ARG, "row tile must be 16 or 32");
  if (rtile == 16 && b->model->w.prec == PSWA_PREC_F32)
    return fail(PSWA_E_UNSUPPORTED, "FP32 models use 16-row FP32 tiles only");
  const int lim = rtile == 16 ? b->max_grid_r16 : b->max_grid_r32;
  if (b->grid > lim)
    return fail(PSWA_E_ARG, "the current %d blocks exceed the %d co-resident with %d-row tiles; "
                "regroup first", b->grid, lim, rtile);
  b->rtile = rtile;
  drop_graph(b);
  return PSWA_OK;
}

int pswa_batch_rtile(const pswa_batch* b) { return b ? b->rtile : -1; }

pswa_status pswa_batch_capture(pswa_batch* b, void* stream) {
  if (!b) return fail(PSWA_E_ARG, "batch is null");
  if (prof_on()) return fail(PSWA_E_ARG, "turn the kernel timer off before capturing");
  (void)stream;
  drop_graph(b);
  // capture on a private stream (the null stream cannot be captured)
  hipStream_t cs;
  PSWA_HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  pswa_status st = PSWA_OK;
  if (e == hipSuccess) {
    st = run(b, cs);
    e = hipStreamEndCapture(cs, &g);
  }
  if (e == hipSuccess && st == PSWA_OK) e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  (void)hipStreamDestroy(cs);
  if (st != PSWA_OK) return st;
  if (e != hipSuccess) {
    b->graph = nullptr;
    return fail(PSWA_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
  }
  return PSWA_OK;
}

pswa_status pswa_batch_autotune(pswa_batch* b, const char* cache_path, int reps, void* stream,
                                int* out_fpg, int* out_bpg, int* out_rtile, float* out_ms) {
  if (!b || !out_fpg || !out_bpg || !out_rtile || !out_ms) return fail(PSWA_E_ARG, "null argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const pswa_model* m = b->model;
  const NetDims& x = m->x;
  const int n = (int)b->finfo.size();
  // cache key: device, model shape and precision, frame mix
  int dev = 0;
  hipDeviceProp_t prop;
  PSWA_HIP_TRY(hipGetDevice(&dev));
  PSWA_HIP_TRY(hipGetDeviceProperties(&prop, dev));
  std::ostringstream key;
  key << prop.gcnArchName << "|L" << x.L << ".d" << x.d << ".h" << x.heads << ".r" << x.r
      << ".F" << x.F << ".C" << x.C << ".p" << m->w.prec << ".c" << x.cycle;
  if (x.cg) key << ".g" << x.cg << "x" << x.cd << "x" << x.cL << "x" << x.cFg;
  key << "|";
  for (const FrameInfo& f : b->finfo) key << f.H << "x" << f.W << (f.n_prev ? "P" : "I") << ",";
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    const std::string k = "{\"key\": \"" + key.str() + "\"";
    while (std::getline(in, line)) {
      if (line.compare(0, k.size(), k) != 0) continue;
      int f = 0, g = 0, r = 0, sa = 0;
      float ms = 0;
      if (std::sscanf(line.c_str() + k.size(),
                      ", \"frames_per_group\": %d, \"blocks_per_group\": %d, \"rtile\": %d, "
                      "\"attn_staged\": %d, \"ms\": %f", &f, &g, &r, &sa, &ms) == 5 &&
          (r == 16 || r == 32) && (r == 32 || m->w.prec) && (sa == 0 || sa == 1)) {
        const int r_old = b->rtile;
        b->rtile = r;
        b->attn_staged = staged_ok(m) ? sa : 0;
        const pswa_status s2 = apply_groups(b, f, g, st);
        if (s2 != PSWA_OK) {  // a stale entry (another device limit): retune
          b->rtile = r_old;
          continue;
        }
        *out_fpg = b->fpg;
        *out_bpg = b->bpg;
        *out_rtile = r;
        *out_ms = ms;
        return PSWA_OK;
      }
    }
  }
  // time a window of the widest global steps for each candidate
  const int w = std::min(b->T, 24);
  const int t0 = std::max(0, b->T / 2 - w / 2);
  hipEvent_t e0, e1;
  PSWA_HIP_TRY(hipEventCreate(&e0));
  PSWA_HIP_TRY(hipEventCreate(&e1));
  float best = 1e30f;
  auto time_it = [&](int r, float* med) -> pswa_status {
    PersistArgs P = persist_args(b);
    P.t_begin = t0;
    P.t_end = t0 + w;
    P.trace = nullptr;
    std::vector<float> t;
    for (int i = 0; i <= std::max(1, reps); ++i) {
      zero_ints(b->ctl, 3, st);
      zero_ints(b->bars, (int)b->groups.size() * kBarStride, st);
      PSWA_HIP_TRY(hipEventRecord(e0, st));
      launch_persistent(P, x, m->w.prec, r, b->grid, st);
      PSWA_HIP_TRY(hipEventRecord(e1, st));
      PSWA_HIP_TRY(hipEventSynchronize(e1));
      float ms = 0;
      PSWA_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      if (i > 0) t.push_back(ms);  // the first run warms up
      // a candidate already 3x slower than the best is not timed further
      if (ms > 3.0f * best) {
        if (t.empty()) t.push_back(ms);
        break;
      }
    }
    int ab = 0;
    PSWA_HIP_TRY(hipMemcpy(&ab, b->ctl + 1, sizeof ab, hipMemcpyDeviceToHost));
    std::sort(t.begin(), t.end());
    *med = ab ? 1e30f : t[t.size() / 2];
    return PSWA_OK;
  };
  // (frames per group, blocks per group): powers of two (and all frames),
  // using at least a sixteenth of the co-resident blocks, for each row tile
  std::vector<int> fpgs;
  for (int f = 1; f < n; f *= 2) fpgs.push_back(f);
  fpgs.push_back(n);
  int bf = b->fpg, bb = b->bpg, br = b->rtile;
  const std::vector<int> rts = m->w.prec == PSWA_PREC_F32 ? std::vector<int>{32}
                                                          : std::vector<int>{32, 16};
  for (int r : rts) {
    const int lim = r == 16 ? b->max_grid_r16 : b->max_grid_r32;
    // regroup within the limit of this row tile before switching to it
    if (b->grid > lim && apply_groups(b, n, std::min(lim, 8), st) != PSWA_OK) continue;
    b->rtile = r;
    for (int f : fpgs)
      for (int g = lim; g >= 2; g /= 2) {
        const int ng = (n + f - 1) / f;
        if ((long)ng * g > lim || ng * g < std::min(16, lim / 16)) continue;
        if (apply_groups(b, f, g, st) != PSWA_OK) continue;
        float med = 0;
        const pswa_status ts = time_it(r, &med);
        if (ts != PSWA_OK) return ts;
        if (med < best) {
          best = med;
          bf = f;
          bb = g;
          br = r;
        }
      }
  }
  // the winner (a grouping valid for its row tile)
  if (b->grid > (br == 16 ? b->max_grid_r16 : b->max_grid_r32))
    (void)apply_groups(b, n, 1, st);
  b->rtile = br;
  pswa_status gs = apply_groups(b, bf, bb, st);
  if (gs != PSWA_OK) return gs;
  // the attention form on the winner (wavefront schedule only)
  int bs = b->attn_staged;
  if (staged_ok(b->model)) {
    for (int sa : {0, 1}) {
      if (sa == bs) continue;
      const int keep = b->attn_staged;
      b->attn_staged = sa;
      float med = 0;
      const pswa_status ts = time_it(br, &med);
      if (ts != PSWA_OK) return ts;
      if (med < best) {
        best = med;
        bs = sa;
      } else {
        b->attn_staged = keep;
      }
    }
    b->attn_staged = bs;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (best >= 1e30f) return fail(PSWA_E_HIP, "autotune: every candidate aborted");
  drop_graph(b);
  *out_fpg = bf;
  *out_bpg = bb;
  *out_rtile = br;
  *out_ms = best * float(b->T) / float(w);  // whole-run estimate
  if (cache_path) {
    std::ofstream o(cache_path, std::ios::app);
    o << "{\"key\": \"" << key.str() << "\", \"frames_per_group\": " << bf
      << ", \"blocks_per_group\": " << bb << ", \"rtile\": " << br
      << ", \"attn_staged\": " << b->attn_staged << ", \"ms\": " << *out_ms << "}\n";
  }
  return PSWA_OK;
}

pswa_status pswa_batch_run(pswa_batch* b, void* stream) {
  if (!b) return fail(PSWA_E_ARG, "batch is null");
  return run(b, static_cast<hipStream_t>(stream));
}

pswa_status pswa_batch_check(pswa_batch* b, void* stream) {
  if (!b) return fail(PSWA_E_ARG, "batch is null");
  hipStream_t st = static_cast<hipStream_t>(stream);
  int ctl[3] = {0, 0, 0};
  PSWA_HIP_TRY(hipMemcpyAsync(ctl, b->ctl, sizeof ctl, hipMemcpyDeviceToHost, st));
  PSWA_HIP_TRY(hipStreamSynchronize(st));
  if (ctl[1]) return fail(PSWA_E_HIP, "persistent decode aborted: a grid barrier wait timed out");
  if (ctl[2]) return fail(PSWA_E_NUMERIC, "non-finite mean or scale produced");
  return PSWA_OK;
}

pswa_status pswa_batch_outputs(pswa_batch* b, int f, int32_t* d_latents_out, float* d_mean,
                               float* d_scale, float* d_bits, int32_t* d_cdf_center,
                               uint16_t* d_cdf_index, double* h_total_bits, void* stream) {
  if (!b) return fail(PSWA_E_ARG, "batch is null");
  if (f < 0 || f >= (int)b->finfo.size()) return fail(PSWA_E_ARG, "frame %d out of range", f);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t C = b->model->x.C;
  const size_t o = (size_t)b->finfo[f].off * C;
  const size_t n = (size_t)b->finfo[f].H * b->finfo[f].W * C;
  auto cp = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    return dst ? hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st) : hipSuccess;
  };
  PSWA_HIP_TRY(cp(d_latents_out, b->ydec + o, n * sizeof(int32_t)));
  PSWA_HIP_TRY(cp(d_mean, b->mean + o, n * sizeof(float)));
  PSWA_HIP_TRY(cp(d_scale, b->scale + o, n * sizeof(float)));
  PSWA_HIP_TRY(cp(d_bits, b->bits + o, n * sizeof(float)));
  PSWA_HIP_TRY(cp(d_cdf_center, b->center + o, n * sizeof(int32_t)));
  PSWA_HIP_TRY(cp(d_cdf_index, b->index + o, n * sizeof(uint16_t)));
  if (h_total_bits) {
    const pswa_status s = pswa_batch_check(b, stream);
    if (s != PSWA_OK) return s;
    return finish_sum(b->bits + o, n, b->sum, b->ctl + 2, h_total_bits, st);
  }
  return PSWA_OK;
}

pswa_status pswa_batch_set_spin_limit(pswa_batch* b, int64_t spins) {
  if (!b) return fail(PSWA_E_ARG, "batch is null");
  if (spins < 0) return fail(PSWA_E_ARG, "spin limit must be >= 0");
  b->spin_limit = long(spins);
  drop_graph(b);
  return PSWA_OK;
}

pswa_status pswa_batch_set_xcd_barrier(pswa_batch* b, int on) {
  if (!b) return fail(PSWA_E_ARG, "batch is null");
  b->xcd_local = on ? 1 : 0;
  drop_graph(b);
  return PSWA_OK;
}

pswa_status pswa_batch_set_attention(pswa_batch* b, int staged) {
  if (!b) return fail(PSWA_E_ARG, "batch is null");
  if (staged && !staged_ok(b->model))
    return fail(PSWA_E_UNSUPPORTED,
                "LDS-staged window tiles serve the wavefront schedule only");
  b->attn_staged = staged ? 1 : 0;
  drop_graph(b);
  return PSWA_OK;
}

int pswa_batch_attention(const pswa_batch* b) { return b ? b->attn_staged : -1; }

pswa_status pswa_batch_trace(pswa_batch* b, int64_t* d_trace, int n) {
  if (!b) return fail(PSWA_E_ARG, "batch is null");
  if (n < 0 || (n > 0 && !d_trace)) return fail(PSWA_E_ARG, "bad trace buffer");
  b->trace = reinterpret_cast<long long*>(d_trace);
  b->trace_len = n;
  drop_graph(b);
  return PSWA_OK;
}

void pswa_batch_destroy(pswa_batch* b) { delete b; }

}  // extern "C"
