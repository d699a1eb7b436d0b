// FP64 matrix-core GEMM for gfx950.
//
// C = beta*C + sum_ph alpha_ph * op(A_ph) * op(B_ph) over one or two "phases", batched over
// grid.z (independent chains) and grid.y (sub-problems).  Operands are strided quadrant views
// (common.h), which lets one kernel read the block-plus-arrow operands of the BTA sweeps
// ([L_B; L_C], the augmented inverse [[Z_D, Z_C^T]; [Z_C, Z_T]]) without copies.
//
// Tiling: a 256-thread workgroup owns a 64 x 64 tile of C; each of its four wavefronts owns
// a 32 x 32 quarter as 2 x 2 fragments of v_mfma_f64_16x16x4.  K advances 16 at a time
// through LDS with the next tile prefetched into registers.  On this instruction lane l holds
// A[l%16][l/16], B[l/16][l%16] and D[l/16 + 4v][l%16] (v = 0..3); the kernel feeds the
// B-fragment as the instruction's A operand so that each lane's results lie along a column of
// C and 16 consecutive lanes write 16 consecutive doubles.
#include "common.h"
#include "profile.h"
#include <climits>
#include <cmath>
#include <algorithm>

namespace adelia {

namespace {

constexpr int BM = 64, BN = 64, BK = 32;
constexpr int LDS_ROW = BM + 4;  // padded row (doubles); keeps 16-byte alignment

struct QuadSel {
  const double* p;
  long long sr, sc;
};

__device__ __forceinline__ QuadSel pick(const View& v, int q, int z, int y) {
  // all four quadrants are read (uniform kernel arguments) and selected per lane; an indexed
  // access would make the compiler spill the argument block to scratch
  const bool hi = (q & 1) != 0, right = (q & 2) != 0;
  const double* p01 = hi ? v.p[1] : v.p[0];
  const double* p23 = hi ? v.p[3] : v.p[2];
  const long long sr01 = hi ? v.sr[1] : v.sr[0], sr23 = hi ? v.sr[3] : v.sr[2];
  const long long sc01 = hi ? v.sc[1] : v.sc[0], sc23 = hi ? v.sc[3] : v.sc[2];
  const long long zs01 = hi ? v.zs[1] : v.zs[0], zs23 = hi ? v.zs[3] : v.zs[2];
  const long long ys01 = hi ? v.ys[1] : v.ys[0], ys23 = hi ? v.ys[3] : v.ys[2];
  QuadSel s;
  s.sr = right ? sr23 : sr01;
  s.sc = right ? sc23 : sc01;
  const long long zs = right ? zs23 : zs01, ys = right ? ys23 : ys01;
  s.p = (right ? p23 : p01) + (long long)z * zs + (long long)y * ys;
  return s;
}

__device__ __forceinline__ double* elem_ptr(const View& v, int r, int c, int z, int y) {
  const bool rb = r >= v.rs, cb = c >= v.cs;
  const int q = (rb ? 1 : 0) + (cb ? 2 : 0);
  QuadSel s = pick(v, q, z, y);
  const int rr = rb ? r - v.rs : r;
  const int cc = cb ? c - v.cs : c;
  return const_cast<double*>(s.p + rr * s.sr + cc * s.sc);
}

// Whole region [r0, r0+R) x [c0, c0+Cn) inside one quadrant?  Returns quadrant or -1.
__device__ __forceinline__ int uniform_quad(const View& v, int r0, int R, int c0, int Cn) {
  const bool rb0 = r0 >= v.rs, rb1 = (r0 + R - 1) >= v.rs;
  const bool cb0 = c0 >= v.cs, cb1 = (c0 + Cn - 1) >= v.cs;
  if (rb0 != rb1 || cb0 != cb1) return -1;
  return (rb0 ? 1 : 0) + (cb0 ? 2 : 0);
}

__device__ __forceinline__ bool tri_zero(int tri, int r, int c) {
  return (tri == TRI_LOWER && c > r) || (tri == TRI_UPPER && r > c);
}

// Tile loads.  A BM x BK tile of logical A (and a BK x BN tile of logical B) goes through 8
// registers per thread.  Fast paths (tile inside one quadrant and in bounds) use 16-byte loads
// along the contiguous dimension; mode records the thread -> element mapping for the LDS store:
//   0: pairs along M (N for B), 1: pairs along K, 2: generic scalar (M/N fastest).
struct TileRegs {
  double v[8];
  int mode;
};

__device__ __forceinline__ bool vec_ok(const double* base, long long other_stride) {
  return ((reinterpret_cast<uintptr_t>(base) & 15) == 0) && ((other_stride & 1) == 0);
}

__device__ __forceinline__ void load_a(const View& A, int M, int K, int m0, int k0, int tri,
                                       double alpha, int z, int y, TileRegs& t) {
  const int tid = threadIdx.x;
  const bool inb = (m0 + BM <= M) && (k0 + BK <= K);
  const int q = inb ? uniform_quad(A, m0, BM, k0, BK) : -1;
  if (q >= 0) {
    QuadSel s = pick(A, q, z, y);
    const int mo = (q & 1) ? m0 - A.rs : m0;
    const int ko = (q & 2) ? k0 - A.cs : k0;
    const double* base = s.p + mo * s.sr + ko * s.sc;
    if (s.sr == 1 && vec_ok(base, s.sc)) {
      t.mode = 0;
      const int m = (tid & 31) * 2, kq = tid >> 5;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = kq + 8 * j;
        const double2 v = *reinterpret_cast<const double2*>(base + m + k * s.sc);
        double v0 = v.x, v1 = v.y;
        if (tri) {
          if (tri_zero(tri, m0 + m, k0 + k)) v0 = 0.0;
          if (tri_zero(tri, m0 + m + 1, k0 + k)) v1 = 0.0;
        }
        t.v[2 * j] = alpha * v0;
        t.v[2 * j + 1] = alpha * v1;
      }
      return;
    }
    if (s.sc == 1 && vec_ok(base, s.sr)) {
      t.mode = 1;
      const int k = (tid & 15) * 2, mq = tid >> 4;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int m = mq + 16 * j;
        const double2 v = *reinterpret_cast<const double2*>(base + m * s.sr + k);
        double v0 = v.x, v1 = v.y;
        if (tri) {
          if (tri_zero(tri, m0 + m, k0 + k)) v0 = 0.0;
          if (tri_zero(tri, m0 + m, k0 + k + 1)) v1 = 0.0;
        }
        t.v[2 * j] = alpha * v0;
        t.v[2 * j + 1] = alpha * v1;
      }
      return;
    }
    t.mode = 2;
    const int m = tid & 63, kq = tid >> 6;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = kq + 4 * j;
      double val = base[m * s.sr + k * s.sc];
      if (tri && tri_zero(tri, m0 + m, k0 + k)) val = 0.0;
      t.v[j] = alpha * val;
    }
    return;
  }
  t.mode = 2;
  const int m = tid & 63, kq = tid >> 6;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int k = kq + 4 * j;
    const int gm = m0 + m, gk = k0 + k;
    double val = 0.0;
    if (gm < M && gk < K && !(tri && tri_zero(tri, gm, gk))) val = *elem_ptr(A, gm, gk, z, y);
    t.v[j] = alpha * val;
  }
}

__device__ __forceinline__ void store_a(const TileRegs& t, double (*As)[LDS_ROW]) {
  const int tid = threadIdx.x;
  if (t.mode == 0) {
    const int m = (tid & 31) * 2, kq = tid >> 5;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      *reinterpret_cast<double2*>(&As[kq + 8 * j][m]) = make_double2(t.v[2 * j], t.v[2 * j + 1]);
  } else if (t.mode == 1) {
    const int k = (tid & 15) * 2, mq = tid >> 4;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      As[k][mq + 16 * j] = t.v[2 * j];
      As[k + 1][mq + 16 * j] = t.v[2 * j + 1];
    }
  } else {
    const int m = tid & 63, kq = tid >> 6;
#pragma unroll
    for (int j = 0; j < 8; ++j) As[kq + 4 * j][m] = t.v[j];
  }
}

// Logical B(k, n), tile BK x BN at (k0, n0); stored in LDS as Bs[k][n].
__device__ __forceinline__ void load_b(const View& B, int K, int N, int k0, int n0, int tri, int z,
                                       int y, TileRegs& t) {
  const int tid = threadIdx.x;
  const bool inb = (n0 + BN <= N) && (k0 + BK <= K);
  const int q = inb ? uniform_quad(B, k0, BK, n0, BN) : -1;
  if (q >= 0) {
    QuadSel s = pick(B, q, z, y);
    const int ko = (q & 1) ? k0 - B.rs : k0;
    const int no = (q & 2) ? n0 - B.cs : n0;
    const double* base = s.p + ko * s.sr + no * s.sc;
    if (s.sc == 1 && vec_ok(base, s.sr)) {
      t.mode = 0;
      const int n = (tid & 31) * 2, kq = tid >> 5;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = kq + 8 * j;
        const double2 v = *reinterpret_cast<const double2*>(base + k * s.sr + n);
        double v0 = v.x, v1 = v.y;
        if (tri) {
          if (tri_zero(tri, k0 + k, n0 + n)) v0 = 0.0;
          if (tri_zero(tri, k0 + k, n0 + n + 1)) v1 = 0.0;
        }
        t.v[2 * j] = v0;
        t.v[2 * j + 1] = v1;
      }
      return;
    }
    if (s.sr == 1 && vec_ok(base, s.sc)) {
      t.mode = 1;
      const int k = (tid & 15) * 2, nq = tid >> 4;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int n = nq + 16 * j;
        const double2 v = *reinterpret_cast<const double2*>(base + k + n * s.sc);
        double v0 = v.x, v1 = v.y;
        if (tri) {
          if (tri_zero(tri, k0 + k, n0 + n)) v0 = 0.0;
          if (tri_zero(tri, k0 + k + 1, n0 + n)) v1 = 0.0;
        }
        t.v[2 * j] = v0;
        t.v[2 * j + 1] = v1;
      }
      return;
    }
    t.mode = 2;
    const int n = tid & 63, kq = tid >> 6;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = kq + 4 * j;
      double val = base[k * s.sr + n * s.sc];
      if (tri && tri_zero(tri, k0 + k, n0 + n)) val = 0.0;
      t.v[j] = val;
    }
    return;
  }
  t.mode = 2;
  const int n = tid & 63, kq = tid >> 6;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int k = kq + 4 * j;
    const int gk = k0 + k, gn = n0 + n;
    double val = 0.0;
    if (gk < K && gn < N && !(tri && tri_zero(tri, gk, gn))) val = *elem_ptr(B, gk, gn, z, y);
    t.v[j] = val;
  }
}

__device__ __forceinline__ void store_b(const TileRegs& t, double (*Bs)[LDS_ROW]) {
  const int tid = threadIdx.x;
  if (t.mode == 0) {
    const int n = (tid & 31) * 2, kq = tid >> 5;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      *reinterpret_cast<double2*>(&Bs[kq + 8 * j][n]) = make_double2(t.v[2 * j], t.v[2 * j + 1]);
  } else if (t.mode == 1) {
    const int k = (tid & 15) * 2, nq = tid >> 4;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      Bs[k][nq + 16 * j] = t.v[2 * j];
      Bs[k + 1][nq + 16 * j] = t.v[2 * j + 1];
    }
  } else {
    const int n = tid & 63, kq = tid >> 6;
#pragma unroll
    for (int j = 0; j < 8; ++j) Bs[kq + 4 * j][n] = t.v[j];
  }
}

__device__ __forceinline__ void krange(int mode, int K, int m0, int n0, int& klo, int& khi) {
  klo = 0;
  khi = K;
  switch (mode) {
    case KR_GE_N0: klo = n0; break;
    case KR_LT_N1: khi = min(K, n0 + BN); break;
    case KR_LT_M1: khi = min(K, m0 + BM); break;
    case KR_GE_MAX: klo = max(m0, n0); break;
    default: break;
  }
  klo = (klo / BK) * BK;
  if (klo > K) klo = K;
}

// One phase of the K loop: double-buffered LDS (one barrier per 32-wide K step); the next
// step's tiles travel global -> registers while the current step runs on the matrix cores.
__device__ __forceinline__ void run_phase(const GemmPhase& ph, int M, int N, int m0, int n0,
                                          bool lasty, int z, int y, int wm, int wn, int lane,
                                          double (*As)[BK][LDS_ROW], double (*Bs)[BK][LDS_ROW],
                                          v4d (&acc)[2][2]) {
  const int K = lasty ? ph.Klast : ph.K;
  int klo, khi;
  krange(ph.kmode, K, m0, n0, klo, khi);
  if (klo >= khi) return;
  TileRegs ra, rb;
  load_a(ph.A, M, K, m0, klo, ph.triA, ph.alpha, z, y, ra);
  load_b(ph.B, K, N, klo, n0, ph.triB, z, y, rb);
  __syncthreads();  // the previous phase may still read buffer 0
  store_a(ra, As[0]);
  store_b(rb, Bs[0]);
  __syncthreads();
  int cur = 0;
  for (int k0 = klo; k0 < khi; k0 += BK) {
    const bool more = k0 + BK < khi;
    if (more) {
      load_a(ph.A, M, K, m0, k0 + BK, ph.triA, ph.alpha, z, y, ra);
      load_b(ph.B, K, N, k0 + BK, n0, ph.triB, z, y, rb);
    }
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int kr = kk * 4 + (lane >> 4);
      const double a0 = As[cur][kr][wm + (lane & 15)];
      const double a1 = As[cur][kr][wm + 16 + (lane & 15)];
      const double b0 = Bs[cur][kr][wn + (lane & 15)];
      const double b1 = Bs[cur][kr][wn + 16 + (lane & 15)];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(b0, a0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(b1, a0, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(b0, a1, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(b1, a1, acc[1][1], 0, 0, 0);
    }
    if (more) {
      store_a(ra, As[cur ^ 1]);
      store_b(rb, Bs[cur ^ 1]);
    }
    __syncthreads();
    cur ^= 1;
  }
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2); give every XCD
// a contiguous range of tiles so that neighbouring tiles, which share operand tiles, share an L2.
__device__ __forceinline__ int xcd_remap(int L, int T) {
  const int x = L & 7, idx = L >> 3;
  const int per = T >> 3, rem = T & 7;
  return x * per + min(x, rem) + idx;
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) void gemm_f64_kernel(const GemmArgs args) {
  __shared__ double As[2][BK][LDS_ROW];
  __shared__ double Bs[2][BK][LDS_ROW];
  const int z = blockIdx.z, y = blockIdx.y;
  const bool lasty = (y == (int)gridDim.y - 1);
  const int M = lasty ? args.Mlast : args.M;
  const int N = lasty ? args.Nlast : args.N;
  const int tilesM = (M + BM - 1) / BM, tilesN = (N + BN - 1) / BN;
  int ti, tj;
  if (args.omode == OUT_ALL) {
    const int T = tilesM * tilesN;
    if ((int)blockIdx.x >= T) return;
    const int L = (int)gridDim.x == T ? xcd_remap(blockIdx.x, T) : blockIdx.x;
    ti = L % tilesM;
    tj = L / tilesM;
  } else {
    const int T = tilesM * (tilesM + 1) / 2;
    if ((int)blockIdx.x >= T) return;
    const int L = (int)gridDim.x == T ? xcd_remap(blockIdx.x, T) : blockIdx.x;
    ti = (int)((sqrt(8.0 * L + 1.0) - 1.0) * 0.5);
    while (ti * (ti + 1) / 2 > L) --ti;
    while ((ti + 1) * (ti + 2) / 2 <= L) ++ti;
    tj = L - ti * (ti + 1) / 2;
  }
  const int m0 = ti * BM, n0 = tj * BN;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;

  v4d acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (v4d){0.0, 0.0, 0.0, 0.0};

  run_phase(args.ph[0], M, N, m0, n0, lasty, z, y, wm, wn, lane, As, Bs, acc);
  if (args.nph > 1) run_phase(args.ph[1], M, N, m0, n0, lasty, z, y, wm, wn, lane, As, Bs, acc);

  // epilogue: lane holds C(m0+wm+bi*16 + lane%16, n0+wn+bj*16 + lane/16 + 4v)
  const View& C = args.C;
  const bool full = (m0 + BM <= M) && (n0 + BN <= N);
  const int qc = full ? uniform_quad(C, m0, BM, n0, BN) : -1;
  const double beta = args.beta;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi) {
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm + bi * 16 + (lane & 15);
        const int n = n0 + wn + bj * 16 + (lane >> 4) + 4 * v;
        if (m >= M || n >= N) continue;
        if (args.omode != OUT_ALL && m < n) continue;
        double* dst;
        if (qc >= 0) {
          QuadSel s = pick(C, qc, z, y);
          const int mo = (qc & 1) ? m - C.rs : m;
          const int no = (qc & 2) ? n - C.cs : n;
          dst = const_cast<double*>(s.p + mo * s.sr + no * s.sc);
        } else {
          dst = elem_ptr(C, m, n, z, y);
        }
        double val = acc[bi][bj][v];
        if (beta != 0.0) val += beta * (*dst);
        *dst = val;
        if (args.omode == OUT_LOWER_MIRROR && m > n) *elem_ptr(C, n, m, z, y) = val;
      }
    }
  }
}

}  // namespace


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
  const int tM = (a.M + BM - 1) / BM, tN = (a.N + BN - 1) / BN;
  long long gx;
  if (a.omode == OUT_ALL) {
    gx = (long long)tM * tN;
  } else {
    if (a.M != a.N || a.Mlast != a.Nlast) return -1;
    gx = (long long)tM * (tM + 1) / 2;
  }
  if (gx <= 0) return 0;
  if (gx > INT_MAX) return -1;
  const ProfToken t = prof_begin(s);
  hipLaunchKernelGGL(gemm_f64_kernel, dim3((unsigned)gx, ny, nz), dim3(256), 0, s, a);
  if (t.valid) prof_end_role(t, s, PK_GEMM, (a.tag >= 0 && a.tag < GT_COUNT) ? a.tag : 0,
                            gemm_flops(a, ny) * nz, 0.0);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace adelia
