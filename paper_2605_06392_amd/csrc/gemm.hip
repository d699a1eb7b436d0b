// Device code of the GEMM (tiles, operand staging, pipeline) is in gemm_dev.h; the FP64 GEMM
// kernel and its host launcher are here.
#include "common.h"
#include "gemm_dev.h"
#include "profile.h"

#include <array>
#include <map>
#include <mutex>
#include <vector>
#include <climits>
#include <cmath>
#include <algorithm>

namespace adelia {

using namespace gemm_dev;

namespace {

// LOOP: a capped grid (GemmArgs::maxwg) whose workgroups walk the tiles.
template <bool LOOP, class T>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(1, 2))) void gemm_f64_kernel(const GemmArgs args) {
  __shared__ double As[2][BK][T::LDS_ROW];
  __shared__ double Bs[2][BK][T::LDS_ROW];
  const int z = blockIdx.z, y = blockIdx.y;
  if (z_idle(args.zn, args.step, args.zdiv, z)) return;  // no block of chain z here
  const bool lasty = (y == (int)gridDim.y - 1);
  gemm_walk<LOOP, T>(args, z, y, lasty, blockIdx.x, gridDim.x, As, Bs);
}

// Capped one-phase launches: two tiles per 512-thread workgroup (gemm_walk_dual).
template <class T>
__global__ __launch_bounds__(2 * NT) void gemm_f64_dual_kernel(const GemmArgs args) {
  __shared__ double As[2][2][BK][T::LDS_ROW];
  __shared__ double Bs[2][2][BK][T::LDS_ROW];
  const int z = blockIdx.z, y = blockIdx.y;
  if (z_idle(args.zn, args.step, args.zdiv, z)) return;  // no block of chain z here
  const bool lasty = (y == (int)gridDim.y - 1);
  gemm_walk_dual<T>(args, z, y, lasty, blockIdx.x, gridDim.x, As, Bs);
}

// Tile edge per (block size, role), set by the autotuner (autotune.hip) or a cache file; a
// launch without an entry (or with blk == 0) takes 64.
std::mutex g_tile_mu;
std::map<std::pair<int, int>, int> g_tile;

template <class T>
int launch_gemm_t(const GemmArgs& a, int ny, int nz, hipStream_t s) {
  const int tM = (a.M + T::BM - 1) / T::BM, tN = (a.N + T::BN - 1) / T::BN;
  long long gx;
  if (a.omode == OUT_ALL) {
    gx = (long long)tM * tN;
  } else {
    // lower part of an M x N output with M >= N (a trapezoid when M > N)
    if (a.M < a.N || a.Mlast < a.Nlast) return -1;
    if ((a.Mlast + T::BM - 1) / T::BM > tM || (a.Nlast + T::BN - 1) / T::BN > tN) return -1;
    gx = (long long)tN * (tN + 1) / 2 + (long long)(tM - tN) * tN;
  }
  if (gx <= 0) return 0;
  if (gx > INT_MAX) return -1;
  // the cap counts 64 x 64 tile slots; smaller tiles get proportionally more workgroups
  const long long cap = a.maxwg > 0 ? (long long)a.maxwg * (64 / T::BM) * (64 / T::BN) : 0;
  const bool capped = cap > 0 && gx > cap;
  if (capped) gx = cap < 8 ? 8 : (cap & ~7LL);
  if (gx > INT_MAX) return -1;
  // a capped one-phase launch takes two tiles per workgroup: maxwg tile slots on maxwg / 2 CUs
  const bool dual = capped && a.nph == 1 && gx >= 16;
  const ProfToken t = prof_begin(s);
  if (dual)
    hipLaunchKernelGGL(gemm_f64_dual_kernel<T>, dim3((unsigned)(gx / 16 * 8), ny, nz),
                       dim3(2 * NT), 0, s, a);
  else if (capped)
    hipLaunchKernelGGL((gemm_f64_kernel<true, T>), dim3((unsigned)gx, ny, nz), dim3(NT), 0, s, a);
  else
    hipLaunchKernelGGL((gemm_f64_kernel<false, T>), dim3((unsigned)gx, ny, nz), dim3(NT), 0, s, a);
  if (t.valid) prof_end_role(t, s, PK_GEMM, (a.tag >= 0 && a.tag < GT_COUNT) ? a.tag : 0,
                            gemm_flops(a, ny) * nz, gemm_bytes(a, ny) * nz);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

int tuned_tile(int blk, int tag) {
  if (blk <= 0) return 64;
  std::lock_guard<std::mutex> lock(g_tile_mu);
  auto it = g_tile.find({blk, tag});
  return it == g_tile.end() ? 64 : it->second;
}

void set_tuned_tile(int blk, int tag, int tile) {
  std::lock_guard<std::mutex> lock(g_tile_mu);
  if (tile == 64)
    g_tile.erase({blk, tag});
  else
    g_tile[{blk, tag}] = tile;
}

std::vector<std::array<int, 3>> tuned_tiles() {
  std::lock_guard<std::mutex> lock(g_tile_mu);
  std::vector<std::array<int, 3>> out;
  for (const auto& kv : g_tile) out.push_back({kv.first.first, kv.first.second, kv.second});
  return out;
}

void clear_tuned_tiles() {
  std::lock_guard<std::mutex> lock(g_tile_mu);
  g_tile.clear();
}


// Algorithmic flops of one phase: 2 x the number of (m, n, k) products the mathematics needs,
// given the triangular structure of the operands and the written part of C.
double phase_flops(const GemmPhase& ph, int M, int N, int K, int omode) {
  if (M <= 0 || N <= 0 || K <= 0) return 0.0;
  const bool low = omode != OUT_ALL;
  double s = 0.0;
  if (ph.triA == TRI_UPPER && ph.triB == TRI_LOWER) {
    for (int m = 0; m < M; ++m) {
      const double cols = low ? std::min(N, m + 1) : N;
      // k >= max(m, n): for n <= m this is K - m
      s += cols * std::max(0, K - m);
    }
  } else if (ph.triB == TRI_LOWER) {
    for (int n = 0; n < N; ++n) s += (double)(low ? std::max(0, M - n) : M) * std::max(0, K - n);
  } else if (ph.triB == TRI_UPPER) {
    for (int n = 0; n < N; ++n) s += (double)(low ? std::max(0, M - n) : M) * std::min(K, n + 1);
  } else if (ph.triA == TRI_LOWER) {
    for (int m = 0; m < M; ++m) s += (double)(low ? std::min(N, m + 1) : N) * std::min(K, m + 1);
  } else {
    double outs = 0.0;
    if (low) for (int m = 0; m < M; ++m) outs += std::min(N, m + 1);
    else outs = (double)M * N;
    s = outs * K;
  }
  return 2.0 * s;
}

// Compulsory HBM bytes of one launch: every element of the logical operands read once (half of
// a triangular square operand) and of the written part of C written once (and read once when
// beta != 0); the tile kernels' re-reads of operand tiles are not counted.
double gemm_bytes(const GemmArgs& a, int ny) {
  double e = 0.0;
  for (int y = 0; y < ny; ++y) {
    const bool last = y == ny - 1;
    const int M = last ? a.Mlast : a.M, N = last ? a.Nlast : a.N;
    if (M <= 0 || N <= 0) continue;
    double outs = 0.0;
    if (a.omode != OUT_ALL) {
      for (int m = 0; m < M; ++m) outs += std::min(N, m + 1);
    } else {
      outs = (double)M * N;
    }
    e += outs * (a.beta != 0.0 ? 2.0 : 1.0);
    for (int p = 0; p < a.nph; ++p) {
      const GemmPhase& ph = a.ph[p];
      const int K = last ? ph.Klast : ph.K;
      if (K <= 0) continue;
      e += (double)M * K * (ph.triA && M == K ? 0.5 : 1.0);
      e += (double)K * N * (ph.triB && K == N ? 0.5 : 1.0);
    }
  }
  return 8.0 * e;
}

double gemm_flops(const GemmArgs& a, int ny) {
  double f = 0.0;
  for (int y = 0; y < ny; ++y) {
    const bool last = y == ny - 1;
    const int M = last ? a.Mlast : a.M, N = last ? a.Nlast : a.N;
    for (int p = 0; p < a.nph; ++p)
      f += phase_flops(a.ph[p], M, N, last ? a.ph[p].Klast : a.ph[p].K, a.omode);
  }
  return f;
}

View view_plain(double* p, long long ld, long long zstride, bool trans) {
  View v;
  for (int q = 0; q < 4; ++q) {
    v.p[q] = p;
    v.sr[q] = trans ? ld : 1;
    v.sc[q] = trans ? 1 : ld;
    v.zs[q] = zstride;
    v.ys[q] = 0;
  }
  v.rs = INT_MAX;
  v.cs = INT_MAX;
  return v;
}

View view_rowsplit(double* p0, long long ld0, long long zs0, double* p1, long long ld1,
                   long long zs1, int rsplit, bool trans) {
  View v = view_plain(p0, ld0, zs0, trans);
  // the stored matrix is [X0 (rsplit rows); X1]; a transposed view splits logical columns
  const int q1 = trans ? 2 : 1;
  v.p[q1] = p1;
  v.sr[q1] = trans ? ld1 : 1;
  v.sc[q1] = trans ? 1 : ld1;
  v.zs[q1] = zs1;
  if (trans) v.cs = rsplit; else v.rs = rsplit;
  return v;
}

void view_set_y(View& v, long long ystride) {
  for (int q = 0; q < 4; ++q) v.ys[q] = ystride;
}

int launch_gemm(const GemmArgs& a, int ny, int nz, hipStream_t s) {
  if (a.M <= 0 || a.N <= 0 || ny <= 0 || nz <= 0) return 0;
  if (a.nph < 1 || a.nph > 2) return -1;
  if (ny > 65535 || nz > 65535) return -1;
  // the panel-rows product is formed in place: each tile must cover all columns of its rows
  // (N <= 64), which only the 64 x 64 tile does, so that no tile overwrites columns that another
  // tile of the same rows still reads
  if (a.tag != GT_PROWS && tuned_tile(a.blk, a.tag) == 32) return launch_gemm_t<Tile32>(a, ny, nz, s);
  return launch_gemm_t<Tile64>(a, ny, nz, s);
}

}  // namespace adelia
