// FP64 matrix-core GEMM for gfx950.
//
// C = beta*C + sum_ph alpha_ph * op(A_ph) * op(B_ph) over one or two "phases", batched over
// grid.z (independent chains) and grid.y (sub-problems).  Operands are strided quadrant views
// (common.h), which lets one kernel read the block-plus-arrow operands of the BTA sweeps
// ([L_B; L_C], the augmented inverse [[Z_D, Z_C^T]; [Z_C, Z_T]]) without copies.
//
// Tiling: a 256-thread workgroup owns a BM x BN tile of C (64 x 64, or 32 x 32 for products
// with few tiles, chosen per block size and role by the autotuner); each of its four
// wavefronts owns a quarter as (BM/32) x (BN/32) fragments of v_mfma_f64_16x16x4.  K advances
// 32 at a time through LDS with the next tile prefetched into registers.  On this instruction lane l holds
// A[l%16][l/16], B[l/16][l%16] and D[l/16 + 4v][l%16] (v = 0..3); the kernel feeds the
// B-fragment as the instruction's A operand so that each lane's results lie along a column of
// C and 16 consecutive lanes write 16 consecutive doubles.
#pragma once
#include "common.h"
#include <climits>
#include <cmath>

namespace adelia {
namespace gemm_dev {

constexpr int BK = 32;
// Four wavefronts per tile (eight, with half the MFMAs per wave and K step, measured slower):
// wave w owns rows (w % 2) * WM .. + WM and columns (w / 2) * WN .. + WN, as FI x FJ fragments.
constexpr int NT = 256;

// A square tile shape.  Square, so that the lower-triangular output modes enumerate whole
// tiles of the triangle the same way for every shape.
template <int TILE>
struct Tile {
  static_assert(TILE == 32 || TILE == 64, "tile edge");
  static constexpr int BM = TILE, BN = TILE;
  static constexpr int WM = BM / 2, WN = BN / 2;
  static constexpr int FI = WM / 16, FJ = WN / 16;
  static constexpr int NR = BM * BK / NT;  // staging registers per thread per operand tile
  static constexpr int LDS_ROW = BM + 1;  // odd pitch (doubles): K-contiguous tiles store without bank conflicts
};
using Tile64 = Tile<64>;
using Tile32 = Tile<32>;
// the panel step kernel's update part and the LDS budget of its union use the 64 x 64 tile
constexpr int LDS_ROW = Tile64::LDS_ROW;
constexpr int BM = Tile64::BM, BN = Tile64::BN;

// A view with the chain (z) and sub-problem (y) offsets applied: four quadrant bases and
// strides, formed once per workgroup from the uniform kernel arguments.
struct VP {
  const double* b[4];
  long long sr[4], sc[4];
  int rs, cs;
};

__device__ __forceinline__ VP make_vp(const View& v, int z, int y) {
  VP o;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    o.b[q] = v.p[q] + (long long)z * v.zs[q] + (long long)y * v.ys[q];
    o.sr[q] = v.sr[q];
    o.sc[q] = v.sc[q];
  }
  o.rs = v.rs;
  o.cs = v.cs;
  return o;
}

struct QuadSel {
  const double* p;
  long long sr, sc;
};

// Quadrant q of a view; q may differ between lanes, so the four candidates are selected
// rather than indexed (an indexed access would put the argument block in scratch).
__device__ __forceinline__ QuadSel pick(const VP& v, int q) {
  const bool hi = (q & 1) != 0, right = (q & 2) != 0;
  QuadSel s;
  const double* p01 = hi ? v.b[1] : v.b[0];
  const double* p23 = hi ? v.b[3] : v.b[2];
  const long long sr01 = hi ? v.sr[1] : v.sr[0], sr23 = hi ? v.sr[3] : v.sr[2];
  const long long sc01 = hi ? v.sc[1] : v.sc[0], sc23 = hi ? v.sc[3] : v.sc[2];
  s.p = right ? p23 : p01;
  s.sr = right ? sr23 : sr01;
  s.sc = right ? sc23 : sc01;
  return s;
}

__device__ __forceinline__ double* elem_ptr(const VP& v, int r, int c) {
  const bool rb = r >= v.rs, cb = c >= v.cs;
  QuadSel s = pick(v, (rb ? 1 : 0) + (cb ? 2 : 0));
  const int rr = rb ? r - v.rs : r;
  const int cc = cb ? c - v.cs : c;
  return const_cast<double*>(s.p + rr * s.sr + cc * s.sc);
}

// Whole region [r0, r0+R) x [c0, c0+Cn) inside one quadrant?  Returns quadrant or -1.
__device__ __forceinline__ int uniform_quad(const VP& v, int r0, int R, int c0, int Cn) {
  const bool rb0 = r0 >= v.rs, rb1 = (r0 + R - 1) >= v.rs;
  const bool cb0 = c0 >= v.cs, cb1 = (c0 + Cn - 1) >= v.cs;
  if (rb0 != rb1 || cb0 != cb1) return -1;
  return (rb0 ? 1 : 0) + (cb0 ? 2 : 0);
}

__device__ __forceinline__ bool tri_zero(int tri, int r, int c) {
  return (tri == TRI_LOWER && c > r) || (tri == TRI_UPPER && r > c);
}

// Operand tiles.  A BM x BK tile of logical A (and a BK x BN tile of logical B) goes through NR
// registers per thread.  The lanes of a wavefront walk the operand's contiguous dimension, so
// every load instruction reads 256 or 512 consecutive bytes.
//
// Fast path: while successive K tiles stay inside one quadrant of the view, the loads are
// buffer loads whose per-lane offsets are fixed for the whole stretch; a K step only moves the
// scalar offset.  The buffer descriptor's record count is the quadrant's extent, so lanes of a
// ragged tile that run past the end of the operand read zero instead of faulting; every value
// outside the logical operand is masked when the tile is written to LDS.  Tiles that straddle a
// quadrant boundary take the generic path (per-element addresses clamped into the operand).
typedef const double __attribute__((address_space(1)))* gptr;

template <class T>
struct OpPipe {
  __amdgpu_buffer_rsrc_t rsrc;
  int q;            // quadrant of the current stretch (-1: none yet)
  int mode;         // 0: lanes along M/N, 1: lanes along K
  int kseg;         // K of the stretch's first tile
  long long sK;     // element stride along K inside the quadrant
  unsigned voff[T::NR];
  double v[T::NR];
};

// (row, col) of register j of a tile; rows run along M (or N), cols along K.
template <class T>
__device__ __forceinline__ void tile_pos(int mode, int j, int& r, int& c) {
  const int tid = threadIdx.x & (NT - 1);  // thread within the tile's wavefronts
  const int r0 = tid & (T::BM - 1), c0 = tid / T::BM + (NT / T::BM) * j;
  const int r1 = (tid >> 5) + (NT / 32) * j, c1 = tid & 31;
  r = mode ? r1 : r0;
  c = mode ? c1 : c0;
}

// Quadrant holding the whole tile (tile rows [r0, r0+BM) clipped to R, K range [k0, k0+BK)
// clipped to Kn), or -1 when it straddles a split.  colsfirst: the view's first index is K.
template <class T>
__device__ __forceinline__ int tile_quad(const VP& V, int R, int Kn, int r0, int k0, bool colsfirst) {
  const int r1 = min(r0 + T::BM, R) - 1, k1 = min(k0 + BK, Kn) - 1;
  const int vr0 = colsfirst ? k0 : r0, vr1 = colsfirst ? k1 : r1;
  const int vc0 = colsfirst ? r0 : k0, vc1 = colsfirst ? r1 : k1;
  const bool rb0 = vr0 >= V.rs, rb1 = vr1 >= V.rs, cb0 = vc0 >= V.cs, cb1 = vc1 >= V.cs;
  if (rb0 != rb1 || cb0 != cb1) return -1;
  return (rb0 ? 1 : 0) + (cb0 ? 2 : 0);
}

// Issue the loads of tile (r0, k0).  Nothing reads the loaded registers before store_tile.
template <class T>
__device__ __forceinline__ void load_tile(OpPipe<T>& P, const VP& V, int R, int Kn, int r0, int k0,
                                          bool colsfirst) {
  constexpr int NR = T::NR;
  const int q = tile_quad<T>(V, R, Kn, r0, k0, colsfirst);
  if (q >= 0) {
    if (q != P.q) {  // a new stretch: descriptor and per-lane offsets
      QuadSel s = pick(V, q);
      const int Rv = colsfirst ? Kn : R, Cv = colsfirst ? R : Kn;
      const int rlo = (q & 1) ? V.rs : 0, rhi = (q & 1) ? Rv : min(V.rs, Rv);
      const int clo = (q & 2) ? V.cs : 0, chi = (q & 2) ? Cv : min(V.cs, Cv);
      const long long last = (long long)(rhi - rlo - 1) * s.sr + (long long)(chi - clo - 1) * s.sc;
      const long long bytes = 8 * (last + 1);
      P.rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(s.p), (short)0,
                                                 (int)min(bytes, kMaxOperandBytes), 0x00020000);
      const long long sR = colsfirst ? s.sc : s.sr;
      P.sK = colsfirst ? s.sr : s.sc;
      P.mode = (sR != 1 && P.sK == 1) ? 1 : 0;
      P.kseg = k0;
      const int tr = (colsfirst ? r0 - clo : r0 - rlo), tk = (colsfirst ? k0 - rlo : k0 - clo);
#pragma unroll
      for (int j = 0; j < NR; ++j) {
        int r, c;
        tile_pos<T>(P.mode, j, r, c);
        P.voff[j] = (unsigned)(8 * ((long long)(tr + r) * sR + (long long)(tk + c) * P.sK));
      }
      P.q = q;
    }
    const int soff = (int)(8 * (long long)(k0 - P.kseg) * P.sK);
#pragma unroll
    for (int j = 0; j < NR; ++j) {
      typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
      const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(P.rsrc, (int)P.voff[j], soff, 0);
      P.v[j] = __builtin_bit_cast(double, w);
    }
    return;
  }
  P.q = -1;
  P.mode = 0;
  gptr ptr[NR];
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    int r, c;
    tile_pos<T>(0, j, r, c);
    const int gr = min(r0 + r, R - 1), gc = min(k0 + c, Kn - 1);
    ptr[j] = (gptr)(colsfirst ? elem_ptr(V, gc, gr) : elem_ptr(V, gr, gc));
  }
#pragma unroll
  for (int j = 0; j < NR; ++j) P.v[j] = *ptr[j];
}

// Write a tile to LDS as T[c][r] (K-major).  Tiles inside the operand with no triangle go
// straight through; otherwise what lies outside the operand or on the zero side of a
// triangular operand is written as zero.  tri is in the view's own (row, col) orientation: for
// A that is (m, k), for B it is (k, n).
template <class T>
__device__ __forceinline__ void store_tile(const OpPipe<T>& P, double (*L)[T::LDS_ROW], int R, int Kn,
                                           int r0, int k0, int tri, bool colsfirst) {
  constexpr int NR = T::NR;
  const bool interior = (r0 + T::BM <= R) && (k0 + BK <= Kn) && tri == TRI_NONE;
  if (interior) {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
      int r, c;
      tile_pos<T>(P.mode, j, r, c);
      L[c][r] = P.v[j];
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    int r, c;
    tile_pos<T>(P.mode, j, r, c);
    const int gr = r0 + r, gc = k0 + c;
    bool ok = gr < R && gc < Kn;
    if (tri) ok = ok && !(colsfirst ? tri_zero(tri, gc, gr) : tri_zero(tri, gr, gc));
    L[c][r] = ok ? P.v[j] : 0.0;
  }
}

template <class T>
__device__ __forceinline__ void krange(int mode, int K, int m0, int n0, int& klo, int& khi) {
  klo = 0;
  khi = K;
  switch (mode) {
    case KR_GE_N0: klo = n0; break;
    case KR_LT_N1: khi = min(K, n0 + T::BN); break;
    case KR_LT_M1: khi = min(K, m0 + T::BM); break;
    case KR_GE_MAX: klo = max(m0, n0); break;
    default: break;
  }
  klo = (klo / BK) * BK;
  if (klo > K) klo = K;
}

// One K step on the matrix cores: 8 x FI x FJ MFMAs per wave over a 32-deep slice of the LDS
// tiles.
template <class T>
__device__ __forceinline__ void mfma_step(const double (*As)[T::LDS_ROW],
                                          const double (*Bs)[T::LDS_ROW], int wm, int wn, int lane,
                                          v4d (&acc)[T::FI][T::FJ]) {
#pragma unroll
  for (int kk = 0; kk < BK / 4; ++kk) {
    const int kr = kk * 4 + (lane >> 4);
    double a[T::FI], b[T::FJ];
#pragma unroll
    for (int bi = 0; bi < T::FI; ++bi) a[bi] = As[kr][wm + 16 * bi + (lane & 15)];
#pragma unroll
    for (int bj = 0; bj < T::FJ; ++bj) b[bj] = Bs[kr][wn + 16 * bj + (lane & 15)];
#pragma unroll
    for (int bj = 0; bj < T::FJ; ++bj)
#pragma unroll
      for (int bi = 0; bi < T::FI; ++bi)
        acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[bj], a[bi], acc[bi][bj], 0, 0, 0);
  }
}

// One phase as a software pipeline with a single site per stage (the kernel stays small, which
// matters for short launches).  Iteration t issues the global loads of K tile t, runs tile t-1
// from LDS on the matrix cores, then writes tile t to the other LDS buffer; one barrier per
// iteration.  alpha is applied by the caller to the accumulators.  [s0, s1): the range of the
// tile's K steps to run (all by default).
template <class T>
__device__ __forceinline__ void run_phase(const GemmPhase& ph, int M, int N, int m0, int n0,
                                          bool lasty, int z, int y, int wm, int wn, int lane,
                                          double (*As)[BK][T::LDS_ROW],
                                          double (*Bs)[BK][T::LDS_ROW],
                                          v4d (&acc)[T::FI][T::FJ], int s0 = 0,
                                          int s1 = INT_MAX) {
  const int K = lasty ? ph.Klast : ph.K;
  int klo, khi;
  krange<T>(ph.kmode, K, m0, n0, klo, khi);
  const int nk = max(0, min(klo < khi ? (khi - klo + BK - 1) / BK : 0, s1) - s0);
  klo += s0 * BK;
  const VP A = make_vp(ph.A, z, y), B = make_vp(ph.B, z, y);
  OpPipe<T> pa, pb;
  pa.q = -1;
  pb.q = -1;
  for (int t = 0; t <= nk; ++t) {
    const int k0 = klo + t * BK;
    if (t < nk) {
      load_tile<T>(pa, A, M, K, m0, k0, false);
      load_tile<T>(pb, B, N, K, n0, k0, true);
    }
    if (t > 0) mfma_step<T>(As[(t - 1) & 1], Bs[(t - 1) & 1], wm, wn, lane, acc);
    if (t < nk) {
      store_tile<T>(pa, As[t & 1], M, K, m0, k0, ph.triA, false);
      store_tile<T>(pb, Bs[t & 1], N, K, n0, k0, ph.triB, true);
    }
    __syncthreads();
  }
}

// Addresses of the FI x FJ x 4 C entries of the calling lane: lane holds
// C(m0+wm+bi*16 + lane%16, n0+wn+bj*16 + lane/16 + 4v), clamped into C (out-of-range entries are
// never stored).
template <class T>
__device__ __forceinline__ void tile_c_addr(const VP& C, int M, int N, int m0, int n0, int wm,
                                            int wn, int lane, double* (&cp)[T::FI][T::FJ][4]) {
#pragma unroll
  for (int bi = 0; bi < T::FI; ++bi)
#pragma unroll
    for (int bj = 0; bj < T::FJ; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        cp[bi][bj][v] = elem_ptr(C, min(m0 + wm + bi * 16 + (lane & 15), M - 1),
                                 min(n0 + wn + bj * 16 + (lane >> 4) + 4 * v, N - 1));
}

// C = beta C + acc on the tile (its written part), with cv the values of C read earlier (only
// used when beta != 0; every tile's C is read and written by its own workgroup alone).  The
// mirrored upper triangle of OUT_LOWER_MIRROR: with `stage` (LDS of at least BM x (BN + 1)
// doubles, free, and every thread of the workgroup calling) the tile goes through LDS and its
// transpose is written with the lanes along the columns of the mirrored tile (coalesced);
// without, each lane writes its own transposed entries.
template <class T>
__device__ __forceinline__ void tile_finish(const GemmArgs& args, const VP& C, int M, int N,
                                            int m0, int n0, int wm, int wn, int lane,
                                            double* (&cp)[T::FI][T::FJ][4],
                                            const double (&cv)[T::FI][T::FJ][4],
                                            v4d (&acc)[T::FI][T::FJ], double* stage = nullptr) {
  const double beta = args.beta;
  const bool lowerC = args.omode != OUT_ALL;
  const bool mirror = args.omode == OUT_LOWER_MIRROR;
  const bool staged = mirror && stage != nullptr;
  if (beta != 0.0) {
#pragma unroll
    for (int bi = 0; bi < T::FI; ++bi)
#pragma unroll
      for (int bj = 0; bj < T::FJ; ++bj)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[bi][bj][v] = fma(beta, cv[bi][bj][v], acc[bi][bj][v]);
  }
#pragma unroll
  for (int bi = 0; bi < T::FI; ++bi) {
#pragma unroll
    for (int bj = 0; bj < T::FJ; ++bj) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm + bi * 16 + (lane & 15);
        const int n = n0 + wn + bj * 16 + (lane >> 4) + 4 * v;
        if (m >= M || n >= N) continue;
        if (lowerC && m < n) continue;
        const double val = acc[bi][bj][v];
        *cp[bi][bj][v] = val;
        if (mirror && !staged && m > n) *elem_ptr(C, n, m) = val;
      }
    }
  }
  // a tile with entries below the diagonal (m > n) mirrors them through LDS; the condition is
  // uniform over the workgroup, so are the barriers
  if (staged && m0 + T::BM - 1 > n0) {
    constexpr int P = T::BN + 1;
    __syncthreads();  // the staging area (operand buffers) is free
#pragma unroll
    for (int bi = 0; bi < T::FI; ++bi)
#pragma unroll
      for (int bj = 0; bj < T::FJ; ++bj)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          stage[(wm + bi * 16 + (lane & 15)) * P + wn + bj * 16 + (lane >> 4) + 4 * v] =
              acc[bi][bj][v];
    __syncthreads();
    // entry (row n0 + r, column m0 + c) of the mirrored tile, r fastest across the lanes
    for (int e = threadIdx.x & (NT - 1); e < T::BM * T::BN; e += NT) {
      const int r = e % T::BN, c = e / T::BN;
      const int m = m0 + c, n = n0 + r;
      if (m < M && n < N && m > n) *elem_ptr(C, n, m) = stage[c * P + r];
    }
    __syncthreads();  // the next tile's operand loads reuse the area
  }
}

// C = beta C + acc on the tile at (m0, n0) (its written part), C read now.
template <class T>
__device__ __forceinline__ void tile_store(const GemmArgs& args, int M, int N, int m0, int n0,
                                           int z, int y, int wm, int wn, int lane,
                                           v4d (&acc)[T::FI][T::FJ]) {
  const VP C = make_vp(args.C, z, y);
  double* cp[T::FI][T::FJ][4];
  tile_c_addr<T>(C, M, N, m0, n0, wm, wn, lane, cp);
  double cv[T::FI][T::FJ][4];
  if (args.beta != 0.0) {
#pragma unroll
    for (int bi = 0; bi < T::FI; ++bi)
#pragma unroll
      for (int bj = 0; bj < T::FJ; ++bj)
#pragma unroll
        for (int v = 0; v < 4; ++v) cv[bi][bj][v] = *cp[bi][bj][v];
  }
  tile_finish<T>(args, C, M, N, m0, n0, wm, wn, lane, cp, cv, acc);
}

// One BM x BN output tile at (m0, n0).
template <class T>
__device__ __forceinline__ void gemm_tile(const GemmArgs& args, int M, int N, int m0, int n0,
                                          bool lasty, int z, int y, int wm, int wn, int lane,
                                          double (*As)[BK][T::LDS_ROW],
                                          double (*Bs)[BK][T::LDS_ROW]) {
  // with beta != 0 the reads of C are issued first, so that their latency overlaps the K loop
  // (short-K tiles, such as the rank-64 updates, would otherwise wait for them at the end)
  const VP C = make_vp(args.C, z, y);
  double* cp[T::FI][T::FJ][4];
  tile_c_addr<T>(C, M, N, m0, n0, wm, wn, lane, cp);
  double cv[T::FI][T::FJ][4];
  if (args.beta != 0.0) {
#pragma unroll
    for (int bi = 0; bi < T::FI; ++bi)
#pragma unroll
      for (int bj = 0; bj < T::FJ; ++bj)
#pragma unroll
        for (int v = 0; v < 4; ++v) cv[bi][bj][v] = *cp[bi][bj][v];
  }
  v4d acc[T::FI][T::FJ];
#pragma unroll
  for (int bi = 0; bi < T::FI; ++bi)
#pragma unroll
    for (int bj = 0; bj < T::FJ; ++bj) acc[bi][bj] = (v4d){0.0, 0.0, 0.0, 0.0};
  // acc collects sum_p alpha_p A_p B_p: the products of phase p are accumulated unscaled, the
  // running sum is rescaled by alpha_{p-1} / alpha_p before phase p and by the last alpha at the
  // end (exact for the +-1 used on the sweeps).
  double alpha_prev = 1.0;
  for (int p = 0; p < args.nph; ++p) {
    const double alpha = args.ph[p].alpha;
    if (p > 0) {
      const double sc = alpha_prev / alpha;
#pragma unroll
      for (int bi = 0; bi < T::FI; ++bi)
#pragma unroll
        for (int bj = 0; bj < T::FJ; ++bj) acc[bi][bj] *= sc;
    }
    run_phase<T>(args.ph[p], M, N, m0, n0, lasty, z, y, wm, wn, lane, As, Bs, acc);
    alpha_prev = alpha;
  }
#pragma unroll
  for (int bi = 0; bi < T::FI; ++bi)
#pragma unroll
    for (int bj = 0; bj < T::FJ; ++bj) acc[bi][bj] *= alpha_prev;
  // the two operand buffers of A (2 x BK x (BM + 1) doubles) hold a staged BM x (BN + 1) tile
  static_assert(2 * BK * T::LDS_ROW >= T::BM * (T::BN + 1), "staging area");
  tile_finish<T>(args, C, M, N, m0, n0, wm, wn, lane, cp, cv, acc, &As[0][0][0]);
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2); give every XCD
// a contiguous range of tiles so that neighbouring tiles, which share operand tiles, share an L2.
// With a triangular operand the K range, and so the work, of a tile depends on its row or
// column, and a fixed assignment would hand one XCD the longest tiles of every problem: when the
// ranges are of equal size (T a multiple of 8) the assignment is rotated by `rot` (the problem's
// grid index), so that over a batch every XCD takes every range equally often.
__device__ __forceinline__ int xcd_remap(int L, int T, int rot = 0) {
  const int per = T >> 3, rem = T & 7;
  const int x = rem == 0 ? ((L + rot) & 7) : (L & 7), idx = L >> 3;
  return x * per + min(x, rem) + idx;
}

// K steps of the tile at (m0, n0) in phase ph.
template <class T>
__device__ __forceinline__ int tile_nk(const GemmPhase& ph, bool lasty, int m0, int n0) {
  int klo, khi;
  krange<T>(ph.kmode, lasty ? ph.Klast : ph.K, m0, n0, klo, khi);
  return klo < khi ? (khi - klo + BK - 1) / BK : 0;
}

// run_phase for two tiles in one workgroup: both halves run nkr + 1 pipeline iterations (one
// barrier each), a half whose tile has fewer K steps (or no tile) idles through the rest.
template <class T>
__device__ __forceinline__ void run_phase_locked(const GemmPhase& ph, int M, int N, int m0, int n0,
                                                 bool lasty, int z, int y, int wm, int wn,
                                                 int lane, double (*As)[BK][T::LDS_ROW],
                                                 double (*Bs)[BK][T::LDS_ROW],
                                                 v4d (&acc)[T::FI][T::FJ], bool has, int nkr) {
  const int K = lasty ? ph.Klast : ph.K;
  int klo, khi;
  krange<T>(ph.kmode, K, m0, n0, klo, khi);
  const int nk = has && klo < khi ? (khi - klo + BK - 1) / BK : 0;
  const VP A = make_vp(ph.A, z, y), B = make_vp(ph.B, z, y);
  OpPipe<T> pa, pb;
  pa.q = -1;
  pb.q = -1;
  for (int t = 0; t <= nkr; ++t) {
    const int k0 = klo + t * BK;
    if (t < nk) {
      load_tile<T>(pa, A, M, K, m0, k0, false);
      load_tile<T>(pb, B, N, K, n0, k0, true);
    }
    if (t > 0 && t <= nk) mfma_step<T>(As[(t - 1) & 1], Bs[(t - 1) & 1], wm, wn, lane, acc);
    if (t < nk) {
      store_tile<T>(pa, As[t & 1], M, K, m0, k0, ph.triA, false);
      store_tile<T>(pb, Bs[t & 1], N, K, n0, k0, ph.triB, true);
    }
    __syncthreads();
  }
}

// Tile (ti, tj) of linear index L: column-major over all tiles, or for the lower modes the
// triangle of the top tilesN x tilesN tiles followed by full rows (M >= N).
__device__ __forceinline__ void tile_of(int omode, int L, int tilesM, int tilesN, int T0, int& ti,
                                        int& tj) {
  if (omode == OUT_ALL) {
    ti = L % tilesM;
    tj = L / tilesM;
  } else if (L < T0) {
    ti = (int)((sqrt(8.0 * L + 1.0) - 1.0) * 0.5);
    while (ti * (ti + 1) / 2 > L) --ti;
    while ((ti + 1) * (ti + 2) / 2 <= L) ++ti;
    tj = L - ti * (ti + 1) / 2;
  } else {
    ti = tilesN + (L - T0) / tilesN;
    tj = (L - T0) % tilesN;
  }
}

// Two tiles per 512-thread workgroup (waves 0-3 and 4-7, each half with its own LDS buffers), so
// that every SIMD holds two waves: a capped launch of one-phase products reaches the matrix
// cores' two-wave rate on half as many CUs.  Workgroup b of G takes tile slots b and b + G, then
// b + 2G and b + 3G, ...; with G a multiple of 8 every slot stays on its workgroup's XCD range.
template <class T>
__device__ __forceinline__ void gemm_walk_dual(const GemmArgs& args, int z, int y, bool lasty,
                                               int b, int G, double (*As)[2][BK][T::LDS_ROW],
                                               double (*Bs)[2][BK][T::LDS_ROW]) {
  const int M = lasty ? args.Mlast : args.M;
  const int N = lasty ? args.Nlast : args.N;
  const int tilesM = (M + T::BM - 1) / T::BM, tilesN = (N + T::BN - 1) / T::BN;
  const int h = threadIdx.x >> 8;
  const int lane = threadIdx.x & 63, wave = (threadIdx.x >> 6) & 3;
  const int wm = (wave & 1) * T::WM, wn = (wave >> 1) * T::WN;
  const int T0 = args.omode == OUT_ALL ? 0 : tilesN * (tilesN + 1) / 2;
  const int NTL = args.omode == OUT_ALL ? tilesM * tilesN : T0 + (tilesM - tilesN) * tilesN;
  const bool remap = (G & 7) == 0;
  const GemmPhase& ph = args.ph[0];
  for (int base = b; base < NTL; base += 2 * G) {
    int nkr = 0, ti = 0, tj = 0;
    bool has = false;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int V = base + q * G;
      if (V >= NTL) continue;
      int qi, qj;
      tile_of(args.omode, remap ? xcd_remap(V, NTL, z + y) : V, tilesM, tilesN, T0, qi, qj);
      nkr = max(nkr, tile_nk<T>(ph, lasty, qi * T::BM, qj * T::BN));
      if (q == h) {
        has = true;
        ti = qi;
        tj = qj;
      }
    }
    v4d acc[T::FI][T::FJ];
#pragma unroll
    for (int bi = 0; bi < T::FI; ++bi)
#pragma unroll
      for (int bj = 0; bj < T::FJ; ++bj) acc[bi][bj] = (v4d){0.0, 0.0, 0.0, 0.0};
    run_phase_locked<T>(ph, M, N, ti * T::BM, tj * T::BN, lasty, z, y, wm, wn, lane, As[h], Bs[h],
                        acc, has, nkr);
    if (has) {
#pragma unroll
      for (int bi = 0; bi < T::FI; ++bi)
#pragma unroll
        for (int bj = 0; bj < T::FJ; ++bj) acc[bi][bj] *= ph.alpha;
      tile_store<T>(args, M, N, ti * T::BM, tj * T::BN, z, y, wm, wn, lane, acc);
    }
  }
}

// The tiles of chain z, sub-problem y handled by workgroup slot v of nv: tile v alone, or with
// LOOP tiles v, v + nv, ... (a capped grid; the XCD mapping is kept when nv is a multiple of 8).
template <bool LOOP, class T = Tile64>
__device__ __forceinline__ void gemm_walk(const GemmArgs& args, int z, int y, bool lasty, int v,
                                          int nv, double (*As)[BK][T::LDS_ROW],
                                          double (*Bs)[BK][T::LDS_ROW]) {
  const int M = lasty ? args.Mlast : args.M;
  const int N = lasty ? args.Nlast : args.N;
  const int tilesM = (M + T::BM - 1) / T::BM, tilesN = (N + T::BN - 1) / T::BN;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave & 1) * T::WM, wn = (wave >> 1) * T::WN;
  const int T0 = args.omode == OUT_ALL ? 0 : tilesN * (tilesN + 1) / 2;
  const int NTL = args.omode == OUT_ALL ? tilesM * tilesN : T0 + (tilesM - tilesN) * tilesN;
  if constexpr (LOOP) {
    const bool remap = nv == NTL || (nv & 7) == 0;
    for (int V = v; V < NTL; V += nv) {
      int ti, tj;
      tile_of(args.omode, remap ? xcd_remap(V, NTL, z + y) : V, tilesM, tilesN, T0, ti, tj);
      gemm_tile<T>(args, M, N, ti * T::BM, tj * T::BN, lasty, z, y, wm, wn, lane, As, Bs);
    }
  } else {
    // the grid may cover fewer tiles than the problem has (the first rounds of a launch whose
    // last round is split along K): the first nv tiles
    const int L = xcd_remap(v, nv, z + y);
    if (L >= NTL) return;
    int ti, tj;
    tile_of(args.omode, L, tilesM, tilesN, T0, ti, tj);
    gemm_tile<T>(args, M, N, ti * T::BM, tj * T::BN, lasty, z, y, wm, wn, lane, As, Bs);
  }
}

// ---- two tiles of a row per workgroup (the look-ahead step's update part) ----------------
//
// A kernel that holds one workgroup per CU (the look-ahead step: its panel workgroups need
// 134 KB of LDS) runs one wave per SIMD, so a single tile's K steps leave the matrix cores idle
// while its loads are in flight.  There the update's workgroups take two horizontally adjacent
// tiles (ti, tj) and (ti, tj + 1) of the lower trapezoid at once: the A tile is loaded and read
// from LDS once for both, and every wave has twice the independent matrix-core work per K step.
// For one-phase products whose K range does not depend on the column (KR_FULL, KR_LT_M1) and
// whose B is not triangular.

// Units of the lower trapezoid of a tilesM x tilesN tile grid (M >= N): row ti holds
// min(ti + 1, tilesN) tiles, paired from the left (an odd row ends with a single tile).
// Rows 2p and 2p + 1 of the triangle hold p + 1 units each, so the triangle's first 2q rows
// hold q (q + 1) units and its first 2q + 1 rows (q + 1)^2.
__host__ __device__ inline long long pair_units(int tilesM, int tilesN) {
  const long long q = tilesN / 2;
  const long long tri = (tilesN & 1) ? (q + 1) * (q + 1) : q * (q + 1);
  return tri + (long long)(tilesM - tilesN) * ((tilesN + 1) / 2);
}

// Unit L: row ti, first column tj0 and its tile count (1 or 2).
__device__ __forceinline__ void pair_of(int L, int tilesN, int& ti, int& tj0, int& cnt) {
  const int qn = tilesN / 2;
  const int UT = (tilesN & 1) ? (qn + 1) * (qn + 1) : qn * (qn + 1);
  int len;
  if (L < UT) {
    int q = (int)((sqrt(4.0 * L + 1.0) - 1.0) * 0.5);  // largest q with q (q + 1) <= L
    while (q * (q + 1) > L) --q;
    while ((q + 1) * (q + 2) <= L) ++q;
    if (L < (q + 1) * (q + 1)) {
      ti = 2 * q;
      tj0 = 2 * (L - q * (q + 1));
    } else {
      ti = 2 * q + 1;
      tj0 = 2 * (L - (q + 1) * (q + 1));
    }
    len = ti + 1;
  } else {
    const int uN = (tilesN + 1) / 2;
    ti = tilesN + (L - UT) / uN;
    tj0 = 2 * ((L - UT) % uN);
    len = tilesN;
  }
  cnt = min(2, len - tj0);
}

// One K step of both tiles: per wave 8 x FI x FJ x 2 MFMAs, the A fragments read once.
template <class T>
__device__ __forceinline__ void mfma_step2(const double (*As)[T::LDS_ROW],
                                           const double (*B0)[T::LDS_ROW],
                                           const double (*B1)[T::LDS_ROW], int wm, int wn,
                                           int lane, v4d (&acc0)[T::FI][T::FJ],
                                           v4d (&acc1)[T::FI][T::FJ]) {
#pragma unroll
  for (int kk = 0; kk < BK / 4; ++kk) {
    const int kr = kk * 4 + (lane >> 4);
    double a[T::FI], b0[T::FJ], b1[T::FJ];
#pragma unroll
    for (int bi = 0; bi < T::FI; ++bi) a[bi] = As[kr][wm + 16 * bi + (lane & 15)];
#pragma unroll
    for (int bj = 0; bj < T::FJ; ++bj) {
      b0[bj] = B0[kr][wn + 16 * bj + (lane & 15)];
      b1[bj] = B1[kr][wn + 16 * bj + (lane & 15)];
    }
#pragma unroll
    for (int bj = 0; bj < T::FJ; ++bj)
#pragma unroll
      for (int bi = 0; bi < T::FI; ++bi) {
        acc0[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(b0[bj], a[bi], acc0[bi][bj], 0, 0, 0);
        acc1[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(b1[bj], a[bi], acc1[bi][bj], 0, 0, 0);
      }
  }
}

// run_phase for the tiles at (m0, n0) and (m0, n0 + BN), one pipeline.
template <class T>
__device__ __forceinline__ void run_phase2(const GemmPhase& ph, int M, int N, int m0, int n0,
                                           int z, int wm, int wn, int lane,
                                           double (*As)[BK][T::LDS_ROW],
                                           double (*B0)[BK][T::LDS_ROW],
                                           double (*B1)[BK][T::LDS_ROW],
                                           v4d (&acc0)[T::FI][T::FJ], v4d (&acc1)[T::FI][T::FJ]) {
  const int K = ph.Klast;
  int klo, khi;
  krange<T>(ph.kmode, K, m0, n0, klo, khi);
  const int nk = klo < khi ? (khi - klo + BK - 1) / BK : 0;
  const VP A = make_vp(ph.A, z, 0), B = make_vp(ph.B, z, 0);
  OpPipe<T> pa, pb0, pb1;
  pa.q = -1;
  pb0.q = -1;
  pb1.q = -1;
  for (int t = 0; t <= nk; ++t) {
    const int k0 = klo + t * BK;
    if (t < nk) {
      load_tile<T>(pa, A, M, K, m0, k0, false);
      load_tile<T>(pb0, B, N, K, n0, k0, true);
      load_tile<T>(pb1, B, N, K, n0 + T::BN, k0, true);
    }
    if (t > 0)
      mfma_step2<T>(As[(t - 1) & 1], B0[(t - 1) & 1], B1[(t - 1) & 1], wm, wn, lane, acc0, acc1);
    if (t < nk) {
      store_tile<T>(pa, As[t & 1], M, K, m0, k0, ph.triA, false);
      store_tile<T>(pb0, B0[t & 1], N, K, n0, k0, ph.triB, true);
      store_tile<T>(pb1, B1[t & 1], N, K, n0 + T::BN, k0, ph.triB, true);
    }
    __syncthreads();
  }
}

// The units of chain z handled by workgroup slot v of nv (v, v + nv, ...), a one-phase lower
// product with ny == 1; the XCD mapping is kept when nv covers the units or is a multiple of 8.
template <class T = Tile64>
__device__ __forceinline__ void gemm_walk_pairs(const GemmArgs& args, int z, int v, int nv,
                                                double (*As)[BK][T::LDS_ROW],
                                                double (*B0)[BK][T::LDS_ROW],
                                                double (*B1)[BK][T::LDS_ROW]) {
  const int M = args.Mlast, N = args.Nlast;
  const int tilesM = (M + T::BM - 1) / T::BM, tilesN = (N + T::BN - 1) / T::BN;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave & 1) * T::WM, wn = (wave >> 1) * T::WN;
  const int NU = (int)pair_units(tilesM, tilesN);
  const bool remap = nv == NU || (nv & 7) == 0;
  const GemmPhase& ph = args.ph[0];
  for (int V = v; V < NU; V += nv) {
    int ti, tj0, cnt;
    pair_of(remap ? xcd_remap(V, NU, z) : V, tilesN, ti, tj0, cnt);
    const int m0 = ti * T::BM, n0 = tj0 * T::BN;
    // C is read in the epilogue: reading both tiles' C before the K loop, as gemm_tile does,
    // took the kernel to 256 VGPRs + 68 AGPRs and the split gradient from 33.6 to 34.8 ms
    v4d acc0[T::FI][T::FJ], acc1[T::FI][T::FJ];
#pragma unroll
    for (int bi = 0; bi < T::FI; ++bi)
#pragma unroll
      for (int bj = 0; bj < T::FJ; ++bj) {
        acc0[bi][bj] = (v4d){0.0, 0.0, 0.0, 0.0};
        acc1[bi][bj] = (v4d){0.0, 0.0, 0.0, 0.0};
      }
    if (cnt == 2)
      run_phase2<T>(ph, M, N, m0, n0, z, wm, wn, lane, As, B0, B1, acc0, acc1);
    else
      run_phase<T>(ph, M, N, m0, n0, true, z, 0, wm, wn, lane, As, B0, acc0);
#pragma unroll
    for (int bi = 0; bi < T::FI; ++bi)
#pragma unroll
      for (int bj = 0; bj < T::FJ; ++bj) {
        acc0[bi][bj] *= ph.alpha;
        acc1[bi][bj] *= ph.alpha;
      }
    tile_store<T>(args, M, N, m0, n0, z, 0, wm, wn, lane, acc0);
    if (cnt == 2) tile_store<T>(args, M, N, m0, n0 + T::BN, z, 0, wm, wn, lane, acc1);
  }
}

}  // namespace gemm_dev
}  // namespace adelia
