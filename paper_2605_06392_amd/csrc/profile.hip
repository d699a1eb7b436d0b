// Opt-in per-kernel timing with HIP events (measurement runs only).
//
// While a profile is active every launch made through the instrumented launchers is bracketed
// by two events recorded on the launch's own stream, together with the algorithmic flops and
// HBM bytes the launch is responsible for.  adelia_profile_stop() synchronises and reports the
// totals per kernel.  Inactive (the default) costs one branch per launch.
#include "../../include/adelia.h"
#include "common.h"
#include "internal_api.h"
#include "profile.h"

#include <cstring>
#include <mutex>
#include <string>
#include <vector>

namespace adelia {

namespace {

struct Rec {
  int kind;
  hipEvent_t a, b;
  double flops, bytes;
};

struct ProfState {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t next = 0;
  std::vector<Rec> recs;
  std::mutex mu;
};

ProfState& st() {
  static ProfState s;
  return s;
}

const char* kind_name(int k) {
  switch (k) {
    case PK_GEMM: return "gemm_f64";
    case PK_PANEL: return "potrf_panel";
    case PK_GEMV: return "gemv";
    case PK_ASSEMBLE: return "assemble";
    case PK_TRACE: return "trace";
    case PK_TIP: return "tip";
    case PK_STEP: return "panel_step";
    case PK_WSPARSE: return "w_sparse";
    case PK_GEMM_ROLE0 + 0: return "gemm_f64:other";
    case PK_GEMM_ROLE0 + 1: return "gemm_f64:trailing";
    case PK_GEMM_ROLE0 + 2: return "gemm_f64:trtri";
    case PK_GEMM_ROLE0 + 3: return "gemm_f64:panel_rows";
    case PK_GEMM_ROLE0 + 4: return "gemm_f64:schur_update";
    case PK_GEMM_ROLE0 + 5: return "gemm_f64:si_W";
    case PK_GEMM_ROLE0 + 6: return "gemm_f64:si_ZB";
    case PK_GEMM_ROLE0 + 7: return "gemm_f64:si_ZD";
    case PK_GEMM_SPLIT: return "gemm_f64:split_last_round";
    default: return "other";
  }
}

}  // namespace

bool prof_active() { return st().on; }

ProfToken prof_begin(hipStream_t s) {
  ProfState& P = st();
  ProfToken t{};
  if (!P.on) return t;
  std::lock_guard<std::mutex> g(P.mu);
  if (P.next + 2 > P.pool.size()) return t;  // pool exhausted: stop recording silently
  t.a = P.pool[P.next++];
  t.b = P.pool[P.next++];
  t.valid = true;
  hipEventRecord(t.a, s);
  return t;
}

void prof_end(const ProfToken& t, hipStream_t s, int kind, double flops, double bytes) {
  if (!t.valid) return;
  ProfState& P = st();
  hipEventRecord(t.b, s);
  std::lock_guard<std::mutex> g(P.mu);
  P.recs.push_back(Rec{kind, t.a, t.b, flops, bytes});
}

void prof_end_role(const ProfToken& t, hipStream_t s, int kind, int role, double flops,
                   double bytes, int also) {
  if (!t.valid) return;
  ProfState& P = st();
  hipEventRecord(t.b, s);
  std::lock_guard<std::mutex> g(P.mu);
  P.recs.push_back(Rec{kind, t.a, t.b, flops, bytes});
  P.recs.push_back(Rec{PK_GEMM_ROLE0 + role, t.a, t.b, flops, bytes});
  if (also >= 0 && also < PK_COUNT) P.recs.push_back(Rec{also, t.a, t.b, flops, bytes});
}

}  // namespace adelia

using namespace adelia;

extern "C" {

int adelia_profile_start(adelia_ctx ctx, int max_launches) {
  if (!ctx) return -1;
  if (max_launches < 1) return -2;
  ProfState& P = st();
  std::lock_guard<std::mutex> g(P.mu);
  const size_t need = 2 * (size_t)max_launches;
  while (P.pool.size() < need) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return ADELIA_E_HIP;
    P.pool.push_back(e);
  }
  P.next = 0;
  P.recs.clear();
  P.on = true;
  return 0;
}

int adelia_profile_stop(adelia_ctx ctx, adelia_kernel_stats* out, int max_entries,
                        int* n_entries) {
  if (!ctx) return -1;
  ProfState& P = st();
  std::vector<Rec> recs;
  {
    std::lock_guard<std::mutex> g(P.mu);
    P.on = false;
    recs.swap(P.recs);
  }
  if (hipDeviceSynchronize() != hipSuccess) return ADELIA_E_HIP;
  adelia_kernel_stats acc[PK_COUNT];
  std::memset(acc, 0, sizeof(acc));
  for (int k = 0; k < PK_COUNT; ++k) std::strncpy(acc[k].name, kind_name(k), sizeof(acc[k].name) - 1);
  for (const Rec& r : recs) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return ADELIA_E_HIP;
    adelia_kernel_stats& a = acc[r.kind];
    a.launches += 1;
    a.ms += ms;
    a.flops += r.flops;
    a.bytes += r.bytes;
  }
  int n = 0;
  for (int k = 0; k < PK_COUNT && n < max_entries; ++k)
    if (acc[k].launches > 0) out[n++] = acc[k];
  if (n_entries) *n_entries = n;
  return 0;
}

}  // extern "C"
