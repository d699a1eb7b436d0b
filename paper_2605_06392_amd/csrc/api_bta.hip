// extern "C" entry points: context, batched GEMM and the BTA factor / logdet / solve / selinv.
// Host-side argument validation happens here, before anything is enqueued.
#include "../../include/adelia.h"
#include "common.h"
#include "launchers.h"
#include "internal_api.h"

#include <algorithm>
#include <climits>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>

namespace adelia {

thread_local std::string g_last_error;

void set_last_error(const std::string& s) { g_last_error = s; }

namespace {

__global__ void finalize_info_kernel(int32_t* info, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && info[i] == INT32_MAX) info[i] = 0;
}

// ZT = L^-T L^-1 for one a x a lower factor (ld ld), a <= 64
__global__ __launch_bounds__(64) void lt_gram_inverse_kernel(const double* L, int a, long long ld,
                                                             double* ZT) {
  __shared__ double X[64][65];
  const int tid = threadIdx.x;
  for (int c = tid; c < a; c += 64) {
    for (int r = 0; r < a; ++r) {
      double s = (r == c) ? 1.0 : 0.0;
      for (int m = c; m < r; ++m) s -= L[r + m * ld] * X[m][c];
      X[r][c] = (r >= c) ? s / L[r + r * ld] : 0.0;
    }
  }
  __syncthreads();
  for (int e = tid; e < a * a; e += 64) {
    const int r = e % a, c = e / a;
    double s = 0.0;
    for (int m = (r > c ? r : c); m < a; ++m) s += X[m][r] * X[m][c];
    ZT[r + (long long)c * a] = s;
  }
}

}  // namespace

int launch_finalize_info(int32_t* info, int n, hipStream_t s) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(finalize_info_kernel, dim3((n + 255) / 256), dim3(256), 0, s, info, n);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_lt_gram_inverse(const double* L, int a, long long ld, double* ZT, hipStream_t s) {
  if (a <= 0) return 0;
  if (a > 64) return -1;
  hipLaunchKernelGGL(lt_gram_inverse_kernel, dim3(1), dim3(64), 0, s, L, a, ld, ZT);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace adelia

using namespace adelia;

namespace {

bool aligned8(const void* p) { return ((uintptr_t)p & 7) == 0; }

int check_shape(const adelia_bta_shape& sh) {
  if (sh.n < 1 || sh.b < 1 || sh.a < 0 || sh.a > 64) return ADELIA_E_SHAPE;
  const long long N = (long long)sh.n * sh.b + sh.a;
  if (N > (1LL << 31) - 1) return ADELIA_E_SHAPE;
  if (sh.b > kMaxBlock) return ADELIA_E_SHAPE;  // an operand quadrant would pass 2 GiB
  return 0;
}

struct FactorWs {
  double *Caug, *LCaug, *Taug, *LBC, *S, *ldpart, *zsq;
  int32_t* cnt;
  size_t bytes;
};

FactorWs factor_ws_layout(const adelia_bta_shape& sh, int ap, char* base) {
  const size_t b = sh.b, n = sh.n;
  const int npanel = (sh.b + kPanel - 1) / kPanel;
  size_t off = 0;
  FactorWs w{};
  auto take = [&](size_t count) {
    double* p = base ? reinterpret_cast<double*>(base + off) : nullptr;
    off = align_up(off + count * sizeof(double));
    return p;
  };
  w.Caug = take(n * (size_t)(ap > 0 ? ap : 1) * b);
  w.LCaug = take(n * (size_t)(ap > 0 ? ap : 1) * b);
  w.Taug = take((size_t)(ap > 0 ? ap : 1) * (ap > 0 ? ap : 1));
  w.LBC = take((b + (size_t)(ap > 0 ? ap : 0)) * b);
  w.S = take(b * b);
  w.ldpart = take(n * npanel + 1);
  w.zsq = take(1);
  w.cnt = reinterpret_cast<int32_t*>(take(1));
  w.bytes = off;
  return w;
}

// bta_factor_noalloc works in this array instead of a caller workspace.  Host code never
// passes its name to a kernel (on the host it names a stand-in, not device memory): the
// device address comes from hipGetSymbolAddress, once per device, and is kept per device.
constexpr size_t kNoAllocBytes = ADELIA_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be the current device (nullptr if the
// query failed).
void* scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess && p)
      g_scratch_ptr[device] = p;
    else
      (void)hipGetLastError();  // a failed query must not read as a failed launch later
  }
  return g_scratch_ptr[device];
}

// Arguments 1..10 of bta_factor / bta_factor_noalloc (same numbering).
int check_factor_args(adelia_ctx ctx, const adelia_bta_shape& sh, const double* D,
                      const double* B, const double* C, const double* T, const double* Dinv,
                      const double* rhs, const double* logdet, const int32_t* info) {
  if (!ctx) return -1;
  if (check_shape(sh)) return -2;
  if (!D || !aligned8(D)) return -3;
  if (sh.n > 1 && (!B || !aligned8(B))) return -4;
  if (sh.a > 0 && (!C || !aligned8(C))) return -5;
  if (sh.a > 0 && (!T || !aligned8(T))) return -6;
  if (!Dinv || !aligned8(Dinv)) return -7;
  if (rhs && !aligned8(rhs)) return -8;
  if (!logdet || !aligned8(logdet)) return -9;
  if (!info || ((uintptr_t)info & 3)) return -10;
  if ((long long)sh.n * sh.b > INT_MAX) return ADELIA_E_SHAPE;
  return 0;
}

// The body of bta_factor, on a workspace laid out by factor_ws_layout (checked by the caller).
int factor_enqueue(adelia_ctx ctx, const adelia_bta_shape& sh, double* D, double* B, double* C,
                   double* T, double* Dinv, double* rhs, double* logdet, int32_t* info,
                   const FactorWs& w, hipStream_t s) {
  const int n = sh.n, b = sh.b, a = sh.a;
  const int ap = a + (rhs ? 1 : 0);
  const long long bb = (long long)b * b;
  const long long nb = (long long)n * b;
  int e = 0;
  e |= launch_fill_i32(info, 1, INT32_MAX, s);
  e |= launch_fill_i32(w.cnt, 1, 0, s);
  if (ap > 0) {
    if (a > 0) {
      e |= launch_copy2d(C, a, 0, w.Caug, ap, 0, a, (int)nb, 1, s);
      e |= launch_copy2d(T, a, 0, w.Taug, ap, 0, a, a, 1, s);
    }
    if (rhs) {
      e |= launch_copy2d(rhs, 1, 0, w.Caug + a, ap, 0, 1, (int)nb, 1, s);
      if (a > 0) e |= launch_copy2d(rhs + nb, 1, 0, w.Taug + a, ap, 0, 1, a, 1, s);
      e |= launch_fill(w.Taug + a + (long long)a * ap, 1, 0.0, s);
    }
  }
  if (e) return ADELIA_E_HIP;
  BtaChains c{};
  c.n = n; c.b = b; c.a = a; c.ap = ap; c.nz = 1;
  c.D = D; c.zD = 0; c.slotsD = n;
  c.Bin = B; c.zB = 0; c.slotsB = n > 1 ? n - 1 : 1;
  c.C = w.Caug; c.zC = 0;
  c.LBC = w.LBC; c.zLBC = 0; c.slotsLBC = 1;
  c.T = w.Taug; c.zT = 0;
  c.G = Dinv; c.zG = 0; c.slotsG = n;
  c.ldpart = w.ldpart; c.zLd = 0;
  c.info = info;
  c.cnt = w.cnt;
  c.scratch = w.S; c.zS = 0;
  c.zsq = w.zsq;
  // with the context's streams: look-ahead steps, and each block's inverse on the side stream
  // (every block keeps its L_D and G slot), joined before returning
  const bool side = ctx->has_streams;
  c.invert = !side;
  c.inv_maxwg = side ? ctx->side_maxwg : 0;
  adelia::Lookahead la = ctx->la;
  for (int i = 0; i < n; ++i) {
    int r = bta_forward_block(c, i, s, side ? &la : nullptr);
    if (r) return ADELIA_E_HIP;
    if (side && (hipEventRecord(ctx->fork[i % 3], s) != hipSuccess ||
                 hipStreamWaitEvent(ctx->s2, ctx->fork[i % 3], 0) != hipSuccess ||
                 bta_invert_block(c, i, ctx->s2)))
      return ADELIA_E_HIP;
    // [L_Bi; L_Ci] leave the one-block scratch: L_Bi into B_i, L_Ci (and z_i) into block i of
    // the augmented arrow
    if (i < n - 1 && launch_copy2d(w.LBC, b + ap, 0, B + (long long)i * bb, b, 0, b, b, 1, s))
      return ADELIA_E_HIP;
    if (ap > 0 && launch_copy2d(w.LBC + b, b + ap, 0, w.LCaug + (long long)i * ap * b, ap, 0, ap,
                                b, 1, s))
      return ADELIA_E_HIP;
  }
  if (side && (hipEventRecord(ctx->join, ctx->s2) != hipSuccess ||
               hipStreamWaitEvent(s, ctx->join, 0) != hipSuccess))
    return ADELIA_E_HIP;
  if (bta_tip(c, s)) return ADELIA_E_HIP;
  if (ap > 0) {
    if (a > 0) {
      e |= launch_copy2d(w.LCaug, ap, 0, C, a, 0, a, (int)nb, 1, s);
      e |= launch_copy2d(w.Taug, ap, 0, T, a, 0, a, a, 1, s);
    }
    if (rhs) {
      e |= launch_copy2d(w.LCaug + a, ap, 0, rhs, 1, 0, 1, (int)nb, 1, s);
      if (a > 0) e |= launch_copy2d(w.Taug + a, ap, 0, rhs + nb, 1, 0, 1, a, 1, s);
    }
  }
  const int npanel = (b + kPanel - 1) / kPanel;
  e |= bta_logdet_reduce(w.ldpart, 0, n * npanel + 1, logdet, 0, 1, s);
  e |= launch_zero_upper(D, b, b, bb, n, 0, 1, s);
  e |= launch_zero_upper(Dinv, b, b, bb, n, 0, 1, s);
  e |= launch_finalize_info(info, 1, s);
  return e ? ADELIA_E_HIP : 0;
}

}  // namespace

extern "C" {

int adelia_create(adelia_ctx* ctx, int device) {
  if (!ctx) return -1;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return -2;
  if (hipSetDevice(device) != hipSuccess) return ADELIA_E_HIP;
  adelia_ctx c = new adelia_ctx_s();  // value-initialised: every handle starts null
  c->device = device;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
      cus <= 0)
    cus = 256;
  c->la.cus = cus;
  c->la.slots = cus * gemm_resident_per_cu();
  c->side_maxwg = std::max(16, (5 * cus / 8) & ~15);
  // the device address of bta_factor_noalloc's static scratch, taken here with the device
  // current (null if the query fails: that entry point then returns ADELIA_E_HIP)
  c->noalloc_scratch = scratch_address(device);
  // a GEMM tile table cached by an earlier autotuning run
  tune_load_env();
  bool ok = hipStreamCreateWithFlags(&c->s2, hipStreamNonBlocking) == hipSuccess &&
            hipStreamCreateWithFlags(&c->la.ts, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&c->join, hipEventDisableTiming) == hipSuccess;
  for (int e = 0; e < 3 && ok; ++e)
    ok = hipEventCreateWithFlags(&c->fork[e], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&c->la.pdone[e], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&c->la.tdone[e], hipEventDisableTiming) == hipSuccess;
  c->has_streams = ok;
  *ctx = c;
  return 0;
}

int adelia_destroy(adelia_ctx ctx) {
  if (!ctx) return 0;
  if (ctx->s2) hipStreamSynchronize(ctx->s2);
  if (ctx->la.ts) hipStreamSynchronize(ctx->la.ts);
  for (int e = 0; e < 3; ++e) {
    if (ctx->fork[e]) hipEventDestroy(ctx->fork[e]);
    if (ctx->la.pdone[e]) hipEventDestroy(ctx->la.pdone[e]);
    if (ctx->la.tdone[e]) hipEventDestroy(ctx->la.tdone[e]);
  }
  if (ctx->join) hipEventDestroy(ctx->join);
  if (ctx->s2) hipStreamDestroy(ctx->s2);
  if (ctx->la.ts) hipStreamDestroy(ctx->la.ts);
  delete ctx;
  return 0;
}

const char* adelia_strerror(int code) {
  switch (code) {
    case ADELIA_OK: return "success";
    case ADELIA_E_SHAPE: return "inconsistent or unsupported sizes";
    case ADELIA_E_WORKSPACE: return "workspace too small or misaligned";
    case ADELIA_E_HIP: return "HIP runtime call failed";
    case ADELIA_E_UNSUPPORTED: return "unsupported request";
    case ADELIA_E_STATE: return "no saved forward pass for this workspace";
    default: return code < 0 && code > -100 ? "invalid argument" : "unknown error";
  }
}

const char* adelia_version(void) { return "adelia-gfx950 0.1"; }

const char* adelia_last_error(void) { return g_last_error.c_str(); }

int adelia_dgemm(adelia_ctx ctx, int transA, int transB, int M, int N, int K, double alpha,
                 const double* A, int lda, long long strideA, const double* B, int ldb,
                 long long strideB, double beta, double* C, int ldc, long long strideC,
                 int batch, int uplo, void* stream) {
  if (!ctx) return -1;
  if (transA != 0 && transA != 1) return -2;
  if (transB != 0 && transB != 1) return -3;
  if (M < 0) return -4;
  if (N < 0) return -5;
  if (K < 0) return -6;
  if (M == 0 || N == 0 || batch == 0) return 0;
  if (K > 0 && (!A || !aligned8(A))) return -8;
  if (lda < (transA ? K : M) || lda < 1) return -9;
  if (K > 0 && (!B || !aligned8(B))) return -11;
  if (ldb < (transB ? N : K) || ldb < 1) return -12;
  if (!C || !aligned8(C)) return -15;
  if (ldc < M) return -16;
  if (batch < 0 || batch > 65535) return -18;
  if (uplo != 0 && uplo != 1) return -19;
  if (uplo == 1 && M != N) return ADELIA_E_SHAPE;
  // each operand is one quadrant of the tile kernel's views: its byte extent must fit the
  // 32-bit buffer range
  auto extent = [](long long rows, long long cols, long long ld) {
    return 8 * ((rows - 1) + (cols - 1) * ld + 1);
  };
  if ((K > 0 && (extent(transA ? K : M, transA ? M : K, lda) > kMaxOperandBytes ||
                 extent(transB ? N : K, transB ? K : N, ldb) > kMaxOperandBytes)) ||
      extent(M, N, ldc) > kMaxOperandBytes)
    return ADELIA_E_SHAPE;
  GemmArgs g{};
  g.nph = 1;
  g.ph[0].A = view_plain(const_cast<double*>(A), lda, strideA, transA == 1);
  g.ph[0].B = view_plain(const_cast<double*>(B), ldb, strideB, transB == 1);
  g.ph[0].K = g.ph[0].Klast = K;
  g.ph[0].kmode = KR_FULL;
  g.ph[0].alpha = alpha;
  g.C = view_plain(C, ldc, strideC);
  g.M = g.Mlast = M;
  g.N = g.Nlast = N;
  g.beta = beta;
  g.omode = uplo ? OUT_LOWER : OUT_ALL;
  if (K == 0) {
    // C = beta*C: run with a zero phase
    g.ph[0].K = g.ph[0].Klast = 0;
  }
  return launch_gemm(g, 1, batch, (hipStream_t)stream) ? ADELIA_E_HIP : 0;
}

size_t adelia_bta_workspace_bytes(adelia_bta_shape sh, int which) {
  if (check_shape(sh)) return 0;
  size_t need = 256;
  if (which & ADELIA_WS_FACTOR) {
    FactorWs w = factor_ws_layout(sh, sh.a + 1, nullptr);
    if (w.bytes > need) need = w.bytes;
  }
  if (which & ADELIA_WS_SOLVE) {
    size_t s = align_up((size_t)sh.b * sizeof(double)) + align_up((size_t)(sh.n + 1) * sizeof(double));
    if (s > need) need = s;
  }
  if (which & ADELIA_WS_SELINV) {
    size_t s = align_up(((size_t)sh.b * sh.b + (size_t)sh.a * sh.b) * sizeof(double));
    if (s > need) need = s;
  }
  return need;
}

int bta_factor(adelia_ctx ctx, adelia_bta_shape sh, double* D, double* B, double* C, double* T,
               double* Dinv, double* rhs, double* logdet, int32_t* info, void* ws,
               size_t ws_bytes, void* stream) {
  if (int r = check_factor_args(ctx, sh, D, B, C, T, Dinv, rhs, logdet, info)) return r;
  if (!ws || ((uintptr_t)ws & 255)) return -11;
  const FactorWs w = factor_ws_layout(sh, sh.a + (rhs ? 1 : 0), reinterpret_cast<char*>(ws));
  if (ws_bytes < w.bytes) return ADELIA_E_WORKSPACE;
  return factor_enqueue(ctx, sh, D, B, C, T, Dinv, rhs, logdet, info, w, (hipStream_t)stream);
}

int bta_factor_noalloc(adelia_ctx ctx, adelia_bta_shape sh, double* D, double* B, double* C,
                       double* T, double* Dinv, double* rhs, double* logdet, int32_t* info,
                       void* stream) {
  if (int r = check_factor_args(ctx, sh, D, B, C, T, Dinv, rhs, logdet, info)) return r;
  // the same bound as the workspace query (which assumes a right-hand side), with or without one
  const size_t need = factor_ws_layout(sh, sh.a + 1, nullptr).bytes;
  if (need > kNoAllocBytes) {
    set_last_error("bta_factor_noalloc: this shape needs " + std::to_string(need) +
                   " bytes of scratch; the static scratch holds " +
                   std::to_string(kNoAllocBytes) + " (use bta_factor with a workspace)");
    return ADELIA_E_WORKSPACE;
  }
  if (!ctx->noalloc_scratch) return ADELIA_E_HIP;
  const FactorWs w = factor_ws_layout(sh, sh.a + (rhs ? 1 : 0),
                                      reinterpret_cast<char*>(ctx->noalloc_scratch));
  return factor_enqueue(ctx, sh, D, B, C, T, Dinv, rhs, logdet, info, w, (hipStream_t)stream);
}

int bta_logdet(adelia_ctx ctx, adelia_bta_shape sh, const double* LD, const double* LT,
               double* out, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx) return -1;
  if (check_shape(sh)) return -2;
  if (!LD || !aligned8(LD)) return -3;
  if (sh.a > 0 && (!LT || !aligned8(LT))) return -4;
  if (!out || !aligned8(out)) return -5;
  if (!ws || ((uintptr_t)ws & 255)) return -6;
  if (ws_bytes < (size_t)(sh.n + 1) * sizeof(double)) return ADELIA_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  double* part = reinterpret_cast<double*>(ws);
  const long long bb = (long long)sh.b * sh.b;
  int e = launch_logdiag(LD, sh.b, sh.b, bb, sh.n, part, 0, 0, 1, s);
  if (sh.a > 0) e |= launch_logdiag(LT, sh.a, sh.a, 0, 1, part + sh.n, 0, 0, 1, s);
  else e |= launch_fill(part + sh.n, 1, 0.0, s);
  e |= bta_logdet_reduce(part, 0, sh.n + 1, out, 0, 1, s);
  return e ? ADELIA_E_HIP : 0;
}

int bta_solve(adelia_ctx ctx, adelia_bta_shape sh, const double* Dinv, const double* LB,
              const double* LC, const double* LT, double* x, int flags, void* ws,
              size_t ws_bytes, void* stream) {
  if (!ctx) return -1;
  if (check_shape(sh)) return -2;
  const int n = sh.n, b = sh.b, a = sh.a;
  if (!Dinv || !aligned8(Dinv)) return -3;
  if (n > 1 && (!LB || !aligned8(LB))) return -4;
  if (a > 0 && (!LC || !aligned8(LC))) return -5;
  if (a > 0 && (!LT || !aligned8(LT))) return -6;
  if (!x || !aligned8(x)) return -7;
  if (flags & ~ADELIA_Z_INPUT) return -8;
  if (!ws || ((uintptr_t)ws & 255)) return -9;
  if (ws_bytes < align_up((size_t)b * sizeof(double))) return ADELIA_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  double* y = reinterpret_cast<double*>(ws);
  const long long bb = (long long)b * b;
  const long long nb = (long long)n * b;
  int e = 0;
  if (!(flags & ADELIA_Z_INPUT)) {
    for (int i = 0; i < n; ++i) {
      double* ri = x + (long long)i * b;
      if (i > 0) {
        e |= launch_gemv_n(LB + (long long)(i - 1) * bb, b, 0, x + (long long)(i - 1) * b, 0, 1,
                           ri, 0, 1, y, 0, 1, b, b, 0, -1.0, 1.0, 1, s);
      } else {
        e |= launch_copy2d(ri, b, 0, y, b, 0, b, 1, 1, s);
      }
      e |= launch_gemv_n(Dinv + (long long)i * bb, b, 0, y, 0, 1, nullptr, 0, 0, ri, 0, 1, b, b,
                         1, 1.0, 0.0, 1, s);
      if (a > 0)
        e |= launch_gemv_n(LC + (long long)i * a * b, a, 0, ri, 0, 1, x + nb, 0, 1, x + nb, 0, 1,
                           a, b, 0, -1.0, 1.0, 1, s);
    }
    if (a > 0) e |= launch_tri_small(LT, a, 0, x + nb, 0, a, 0, 1, s);
  }
  if (e) return ADELIA_E_HIP;
  if (a > 0 && launch_tri_small(LT, a, 0, x + nb, 0, a, 1, 1, s)) return ADELIA_E_HIP;
  SolveChains c{};
  c.n = n; c.b = b; c.a = a; c.nz = 1;
  c.G = Dinv; c.zG = 0; c.slotsG = n;
  c.LB = LB; c.zLB = 0; c.slotsLB = n > 1 ? n - 1 : 1; c.ldLB = b; c.sLB = bb;
  c.LC = LC; c.zLC = 0; c.ldLC = a > 0 ? a : 1; c.sLC = (long long)(a > 0 ? a : 1) * b;
  c.z = x; c.zz = 0; c.sz_blk = b; c.sz_elem = 1;
  c.xT = a > 0 ? x + nb : nullptr; c.zxT = 0;
  c.x = x; c.zx = 0;
  c.y = y; c.zy = 0;
  return bta_upper_solve(c, s) ? ADELIA_E_HIP : 0;
}

int bta_selinv(adelia_ctx ctx, adelia_bta_shape sh, const double* Dinv, const double* LB,
               const double* LC, const double* LT, double* ZD, double* ZB, double* ZC,
               double* ZT, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx) return -1;
  if (check_shape(sh)) return -2;
  const int n = sh.n, b = sh.b, a = sh.a;
  if (!Dinv || !aligned8(Dinv)) return -3;
  if (n > 1 && (!LB || !aligned8(LB))) return -4;
  if (a > 0 && (!LC || !aligned8(LC))) return -5;
  if (a > 0 && (!LT || !aligned8(LT))) return -6;
  if (!ZD || !aligned8(ZD)) return -7;
  if (n > 1 && (!ZB || !aligned8(ZB))) return -8;
  if (a > 0 && (!ZC || !aligned8(ZC))) return -9;
  if (a > 0 && (!ZT || !aligned8(ZT))) return -10;
  if (!ws || ((uintptr_t)ws & 255)) return -11;
  if (ws_bytes < ((size_t)b * b + (size_t)a * b) * sizeof(double)) return ADELIA_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  if (a > 0 && launch_lt_gram_inverse(LT, a, a, ZT, s)) return ADELIA_E_HIP;
  SelinvChains c{};
  c.n = n; c.b = b; c.a = a; c.nz = 1;
  c.G = Dinv; c.zG = 0; c.slotsG = n;
  c.LB = LB; c.zLB = 0; c.slotsLB = n > 1 ? n - 1 : 1; c.ldLB = b;
  c.sLB = (long long)b * b;
  c.LC = LC; c.zLC = 0; c.ldLC = a > 0 ? a : 1; c.sLC = (long long)(a > 0 ? a : 1) * b;
  c.ZT = ZT; c.zZT = 0;
  c.ZD = ZD; c.zZD = 0; c.slotsZD = n;
  c.ZB = ZB; c.zZB = 0; c.slotsZB = n > 1 ? n - 1 : 1;
  c.ZC = ZC; c.zZC = 0; c.slotsZC = n;
  c.W = reinterpret_cast<double*>(ws); c.zW = 0; c.slotsW = 1;
  for (int j = n - 1; j >= 0; --j)
    if (selinv_block(c, j, s)) return ADELIA_E_HIP;
  return 0;
}

}  // extern "C"
