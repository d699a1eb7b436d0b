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

// Tiles and lower-mode layout of a launch (as gemm_walk), ny == 1.
struct TileGrid {
  int M, N, tilesM, tilesN, T0, NTL;
};
__device__ __forceinline__ TileGrid tile_grid(const GemmArgs& a, int BM, int BN) {
  TileGrid g;
  g.M = a.Mlast;
  g.N = a.Nlast;
  g.tilesM = (g.M + BM - 1) / BM;
  g.tilesN = (g.N + BN - 1) / BN;
  g.T0 = a.omode == OUT_ALL ? 0 : g.tilesN * (g.tilesN + 1) / 2;
  g.NTL = a.omode == OUT_ALL ? g.tilesM * g.tilesN : g.T0 + (g.tilesM - g.tilesN) * g.tilesN;
  return g;
}

// The last round of a split launch (plan_tail): tile Tm + x / nc of chain z, K steps
// [q nk / nc, (q + 1) nk / nc) of its nk for q = x % nc, alpha applied, stored column-major as
// partial tile ((z R + x / nc) nc + q) of the workspace (R = tiles per chain past Tm).
template <class T>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(1, 2))) void gemm_f64_tail_kernel(
    const GemmArgs args, int Tm, int nc) {
  __shared__ double As[2][BK][T::LDS_ROW];
  __shared__ double Bs[2][BK][T::LDS_ROW];
  const int z = blockIdx.z;
  if (z_idle(args.zn, args.step, args.zdiv, z)) return;
  const TileGrid g = tile_grid(args, T::BM, T::BN);
  const int r = blockIdx.x / nc, q = blockIdx.x - r * nc;
  if (Tm + r >= g.NTL) return;
  int ti, tj;
  tile_of(args.omode, Tm + r, g.tilesM, g.tilesN, g.T0, ti, tj);
  const int m0 = ti * T::BM, n0 = tj * T::BN;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave & 1) * T::WM, wn = (wave >> 1) * T::WN;
  const GemmPhase& ph = args.ph[0];
  const int nk = tile_nk<T>(ph, true, m0, n0);
  v4d acc[T::FI][T::FJ];
#pragma unroll
  for (int bi = 0; bi < T::FI; ++bi)
#pragma unroll
    for (int bj = 0; bj < T::FJ; ++bj) acc[bi][bj] = (v4d){0.0, 0.0, 0.0, 0.0};
  run_phase<T>(ph, g.M, g.N, m0, n0, true, z, 0, wm, wn, lane, As, Bs, acc, q * nk / nc,
               (q + 1) * nk / nc);
  double* P = args.tail.p +
              (((long long)z * (g.NTL - Tm) + r) * nc + q) * (long long)(T::BM * T::BN);
#pragma unroll
  for (int bi = 0; bi < T::FI; ++bi)
#pragma unroll
    for (int bj = 0; bj < T::FJ; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        P[(wn + bj * 16 + (lane >> 4) + 4 * v) * T::BM + wm + bi * 16 + (lane & 15)] =
            acc[bi][bj][v] * ph.alpha;
}

// The split tiles' sums, C = beta C + sum_q P_q with the partials added in chunk order, on the
// written part (lower modes: m >= n; OUT_LOWER_MIRROR also writes the transposed entry).  One
// entry per thread, BM BN / NT workgroups per tile.
template <class T>
__global__ __launch_bounds__(NT) void gemm_f64_fixup_kernel(const GemmArgs args, int Tm, int nc) {
  const int z = blockIdx.z;
  if (z_idle(args.zn, args.step, args.zdiv, z)) return;
  constexpr int E = T::BM * T::BN, PER = E / NT;
  const TileGrid g = tile_grid(args, T::BM, T::BN);
  const int r = blockIdx.x / PER, e = (blockIdx.x - r * PER) * NT + threadIdx.x;
  if (Tm + r >= g.NTL) return;
  int ti, tj;
  tile_of(args.omode, Tm + r, g.tilesM, g.tilesN, g.T0, ti, tj);
  const int m = ti * T::BM + e % T::BM, n = tj * T::BN + e / T::BM;
  if (m >= g.M || n >= g.N) return;
  if (args.omode != OUT_ALL && m < n) return;
  const double* P = args.tail.p + ((long long)z * (g.NTL - Tm) + r) * nc * (long long)E + e;
  double sum = P[0];
#pragma unroll 4
  for (int q = 1; q < nc; ++q) sum += P[(long long)q * E];
  const VP C = make_vp(args.C, z, 0);
  double* cp = elem_ptr(C, m, n);
  const double val = args.beta != 0.0 ? fma(args.beta, *cp, sum) : sum;
  *cp = val;
  if (args.omode == OUT_LOWER_MIRROR && m > n) *elem_ptr(C, n, m) = val;
}

// Tile edge per (block size, role), set by the autotuner (autotune.hip) or a cache file; a
// launch without an entry (or with blk == 0) takes 64.
std::mutex g_tile_mu;
std::map<std::pair<int, int>, int> g_tile;

// Whether to split the last round of an uncapped one-phase launch of gx tiles per chain on nz
// chains (GemmArgs::tail): the tiles take r >= 2 rounds of the device's resident workgroups with
// the last at most half full.  The first r - 1 rounds then hold the first Tm tiles of every chain
// and the remaining R tiles are split into nc K chunks (2 <= nc, R nc within the slots and the
// workspace, at least two K steps per chunk).  At b = 1024 on four chains (the two-sided split)
// this is the Z_D update (544 tiles) and the Schur update (612): 36.5 -> 34.3 ms per gradient.
static bool plan_tail(const GemmArgs& a, long long gx, int nz, int& Tm, int& nc) {
  const TailWs& t = a.tail;
  if (!t.p || t.slots <= 0 || t.tiles <= 0 || a.nph != 1) return false;
  const long long total = gx * nz;
  if (total <= t.slots) return false;
  const long long full = (total / t.slots) * t.slots;
  const long long rem = total - full;
  if (rem == 0 || 2 * rem > t.slots) return false;
  Tm = (int)(full / nz);
  const long long R = (gx - Tm) * nz;
  const long long nk = (a.ph[0].Klast + BK - 1) / BK;
  // at most 8 chunks (b = 1024, split gradient: 34.35 ms against 34.45 with 16 and 34.67 with 4)
  const long long c = std::min<long long>({(long long)t.slots / R, (long long)t.tiles / R, nk / 2,
                                           8LL});
  if (c < 2) return false;
  nc = (int)c;
  return true;
}

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
  int Tm = 0, nc = 0;
  const bool split = !capped && ny == 1 && T::BM == 64 && plan_tail(a, gx, nz, Tm, nc);
  const ProfToken t = prof_begin(s);
  if (dual) {
    hipLaunchKernelGGL(gemm_f64_dual_kernel<T>, dim3((unsigned)(gx / 16 * 8), ny, nz),
                       dim3(2 * NT), 0, s, a);
  } else if (split) {
    hipLaunchKernelGGL((gemm_f64_kernel<false, T>), dim3((unsigned)Tm, 1, nz), dim3(NT), 0, s, a);
    hipLaunchKernelGGL(gemm_f64_tail_kernel<T>, dim3((unsigned)((gx - Tm) * nc), 1, nz), dim3(NT),
                       0, s, a, Tm, nc);
    hipLaunchKernelGGL(gemm_f64_fixup_kernel<T>,
                       dim3((unsigned)((gx - Tm) * (T::BM * T::BN / NT)), 1, nz), dim3(NT), 0, s,
                       a, Tm, nc);
  } else if (capped) {
    hipLaunchKernelGGL((gemm_f64_kernel<true, T>), dim3((unsigned)gx, ny, nz), dim3(NT), 0, s, a);
  } else {
    hipLaunchKernelGGL((gemm_f64_kernel<false, T>), dim3((unsigned)gx, ny, nz), dim3(NT), 0, s, a);
  }
  if (t.valid) prof_end_role(t, s, PK_GEMM, (a.tag >= 0 && a.tag < GT_COUNT) ? a.tag : 0,
                            gemm_flops(a, ny) * nz, gemm_bytes(a, ny) * nz,
                            split ? PK_GEMM_SPLIT : -1);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

int gemm_resident_per_cu() {
  static const int occ = [] {
    int o = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &o, reinterpret_cast<const void*>(&gemm_f64_kernel<false, Tile64>), NT, 0) !=
        hipSuccess)
      o = 0;
    return o;
  }();
  return occ;
}

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
