// Live kernel timing: while enabled, each launch of the library's kernels is
// bracketed by a pair of HIP events on the stream it is launched on, and its
// algorithmic bytes and flops are recorded under the kernel's role. Reading
// waits for the recorded events and sums the elapsed times per role.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/pswa.h"
#include "pswa_internal.h"

namespace pswa {

namespace {

struct Rec {
  int role;
  int ev;  // index of the start event; ev + 1 is the stop event
  double bytes, flops;
};

struct Prof {
  std::mutex mu;
  bool on = false;
  std::vector<hipEvent_t> events;
  size_t used = 0;
  std::vector<Rec> recs;
};

Prof& prof() {
  static Prof p;
  return p;
}

const char* kRoleNames[R_COUNT] = {
    "acc_q_gemm", "acc_attention", "acc_o_gemm", "qkv_gemm", "layer_attention", "o_gemm",
    "gateup_swiglu_gemm", "down_gemm", "head1_gemm", "head2_gemm", "embed_gemm", "acc_kv_gemm",
    "symbol_bits", "gather_symbols", "hyper_embed", "temporal_kv_gemm", "sum", "other",
    "persistent_decode"};

}  // namespace

const char* role_name(int r) { return (r >= 0 && r < R_COUNT) ? kRoleNames[r] : "?"; }

bool prof_on() { return prof().on; }

int prof_begin(hipStream_t s) {
  Prof& p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  if (!p.on) return -1;
  while (p.used + 2 > p.events.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    p.events.push_back(e);
  }
  const int ev = int(p.used);
  p.used += 2;
  if (hipEventRecord(p.events[ev], s) != hipSuccess) return -1;
  return ev;
}

void prof_end(int ev, hipStream_t s, int role, double bytes, double flops) {
  if (ev < 0) return;
  Prof& p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  if (hipEventRecord(p.events[ev + 1], s) != hipSuccess) return;
  p.recs.push_back(Rec{role, ev, bytes, flops});
}

}  // namespace pswa

using namespace pswa;

extern "C" {

pswa_status pswa_profile_enable(int on) {
  Prof& p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  p.on = on != 0;
  if (p.on) {
    p.used = 0;
    p.recs.clear();
  }
  return PSWA_OK;
}

int pswa_profile_roles(void) { return R_COUNT; }

pswa_status pswa_profile_read(int role, char* name, size_t name_cap, double* total_ms,
                              int64_t* launches, double* alg_bytes, double* alg_flops) {
  if (role < 0 || role >= R_COUNT || !total_ms || !launches || !alg_bytes || !alg_flops)
    return PSWA_E_ARG;
  Prof& p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  if (name && name_cap) {
    std::strncpy(name, kRoleNames[role], name_cap - 1);
    name[name_cap - 1] = 0;
  }
  double ms = 0, by = 0, fl = 0;
  int64_t n = 0;
  for (const Rec& r : p.recs) {
    if (r.role != role) continue;
    if (hipEventSynchronize(p.events[r.ev + 1]) != hipSuccess) return PSWA_E_HIP;
    float t = 0.f;
    if (hipEventElapsedTime(&t, p.events[r.ev], p.events[r.ev + 1]) != hipSuccess) return PSWA_E_HIP;
    ms += t;
    by += r.bytes;
    fl += r.flops;
    ++n;
  }
  *total_ms = ms;
  *launches = n;
  *alg_bytes = by;
  *alg_flops = fl;
  return PSWA_OK;
}

}  // extern "C"
