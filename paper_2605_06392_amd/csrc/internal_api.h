// Cross-file host helpers of the C ABI layer.
#pragma once
#include "common.h"
#include <string>

struct adelia_ctx_s {
  int device;
  // streams of the batched sweep (default priority), created with the context: the inversions
  // G_i = L_Di^-1 run on s2 beside the sweep, and the look-ahead updates on la.ts
  bool has_streams;
  hipStream_t s2;
  hipEvent_t fork[3], join;
  adelia::Lookahead la;
  int side_maxwg;
  // device address of the static scratch of bta_factor_noalloc on this device
  void* noalloc_scratch;
};

namespace adelia {
void set_last_error(const std::string& s);
size_t align_up(size_t v);
int launch_finalize_info(int32_t* info, int n, hipStream_t s);
int launch_lt_gram_inverse(const double* L, int a, long long ld, double* ZT, hipStream_t s);
// The GEMM tile table's cache file (autotune.hip): load returns the number of entries read,
// -1 if the file cannot be opened, -2 if it is malformed (nothing is loaded then).
int tune_load_file(const char* path);
int tune_save_file(const char* path);
void tune_load_env();   // from $ADELIA_TUNE_CACHE, if set and readable
void tune_save_env();   // to $ADELIA_TUNE_CACHE, if set
}  // namespace adelia
