// Internal hooks of the opt-in event profiler (profile.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace adelia {

enum ProfKind {
  PK_GEMM = 0, PK_PANEL, PK_GEMV, PK_ASSEMBLE, PK_TRACE, PK_TIP,
  PK_STEP,  // panel k+1 and the trailing update of panel k in one launch
  PK_WSPARSE,  // W_t = B_t (G_t^T G_t) from the sparse B_t
  PK_GEMM_ROLE0,  // + GemmTag: per-role copies of the GEMM statistics
  PK_GEMM_SPLIT = PK_GEMM_ROLE0 + 8,  // copies for the launches whose last round is split
  PK_COUNT
};

struct ProfToken {
  hipEvent_t a, b;
  bool valid;
};

bool prof_active();
ProfToken prof_begin(hipStream_t s);
void prof_end(const ProfToken& t, hipStream_t s, int kind, double flops, double bytes);
// also books the launch under kind `also` when it is >= 0
void prof_end_role(const ProfToken& t, hipStream_t s, int kind, int role, double flops,
                   double bytes, int also = -1);

}  // namespace adelia
