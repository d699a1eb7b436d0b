// Diagonal-block Cholesky pieces of the BTA sweep (Sec. III-A-1, Alg. 1, the chol() steps).
//
// potrf_panel_kernel: one step of a right-looking blocked Cholesky of a b x b diagonal block
// with panel width 64.  Every workgroup factors the 64 x 64 diagonal tile in registers
// (4 x 4 elements per thread, one barrier per column) together with its inverse; workgroup 0
// writes L_kk, L_kk^-1 and the tile's log-diagonal sum, the others solve their 64-row tile of
// the panel as A_jk * L_kk^-T on the matrix cores.  The trailing update between panels is a
// separate GEMM launch (gemm.hip).
//
// tip_kernel: factors the a x a arrowhead tip after the sweep, finishes the forward solve
// (z_T), and forms Z_T = L_T^-T L_T^-1 and x_T = L_T^-T z_T for the backward pass.
#include "common.h"
#include "profile.h"
#include <cmath>

namespace adelia {

namespace {

constexpr int NB = kPanel;      // 64
constexpr int PAD = NB + 4;

struct PanelArgs {
  double* D; long long zD;      // block base (already offset to the block), ld b
  double* G; long long zG;      // inverse block base, ld b
  double* ldp; long long zLd;   // where the tile's sum of log(L_jj) goes
  int32_t* info;                // per chain
  int b, c0;                    // block size, panel column offset
  long long gcol0;              // global column index of the block's first column
};

__global__ __launch_bounds__(256) void potrf_panel_kernel(const PanelArgs P) {
  __shared__ double colb[2][NB];
  __shared__ double pivs[NB];
  __shared__ double xrow[2][NB];
  __shared__ double Xs[NB][PAD];   // Xs[k][n] = Linv(n, k)  (B operand, k-major)
  __shared__ double As[NB][PAD];   // As[k][m] = A(m, k)
  const int tid = threadIdx.x;
  const int z = blockIdx.z;
  const int b = P.b, c0 = P.c0;
  const int w = min(NB, b - c0);
  double* D = P.D + (long long)z * P.zD;
  const int br = tid >> 4, bc = tid & 15;
  const bool active = br >= bc;

  // load my 4x4 block of the diagonal tile (lower part), identity padding past w
  double a[4][4], x[4][4];
#pragma unroll
  for (int ii = 0; ii < 4; ++ii)
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int r = 4 * br + ii, c = 4 * bc + jj;
      double v = 0.0;
      if (r >= c) {
        if (r < w && c < w) v = D[(long long)(c0 + r) + (long long)(c0 + c) * b];
        else if (r == c) v = 1.0;
      }
      a[ii][jj] = v;
      x[ii][jj] = (r == c) ? 1.0 : 0.0;
    }
  // publish column 0 of A and row 0 of X
  if (bc == 0 && active) {
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) colb[0][4 * br + ii] = a[ii][0];
  }
  if (br == 0 && bc == 0) {
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) xrow[0][jj] = x[0][jj];
  }
  __syncthreads();

  // One column per step, one barrier per step.  Masks are folded into the operands so the
  // 4 x 4 updates are branch-free: lc is zero for finished columns (c <= j), lrx is zero for
  // rows r <= j and xj is zero for c > j.
  for (int j = 0; j < NB; ++j) {
    const int cur = j & 1, nxt = cur ^ 1;
    const double djj = colb[cur][j];
    const double piv = sqrt(djj);
    const double invs = 1.0 / piv;
    if (tid == 0) pivs[j] = djj;
    double lr[4], lrx[4], lc[4], xj[4];
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      lr[ii] = colb[cur][4 * br + ii] * invs;
      lrx[ii] = (4 * br + ii > j) ? lr[ii] : 0.0;
    }
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int c = 4 * bc + jj;
      lc[jj] = (c > j) ? colb[cur][c] * invs : 0.0;
      xj[jj] = (c <= j) ? xrow[cur][c] * invs : 0.0;
    }
#pragma unroll
    for (int ii = 0; ii < 4; ++ii)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        a[ii][jj] = fma(-lr[ii], lc[jj], a[ii][jj]);
        x[ii][jj] = fma(-lrx[ii], xj[jj], x[ii][jj]);
      }
    const int jq = j >> 2, jr = j & 3;
    if (bc == jq) {  // finalise column j of L in the owning threads
#pragma unroll
      for (int jj = 0; jj < 4; ++jj)
        if (jj == jr) {
#pragma unroll
          for (int ii = 0; ii < 4; ++ii) a[ii][jj] = (4 * br + ii == j) ? piv : lr[ii];
        }
    }
    if (br == jq) {  // row j of L^-1 is final
#pragma unroll
      for (int ii = 0; ii < 4; ++ii)
        if (ii == jr) {
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) x[ii][jj] = xj[jj];
        }
    }
    if (j + 1 < NB) {
      const int nq = (j + 1) >> 2, nr = (j + 1) & 3;
      if (bc == nq && active) {
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
          if (jj == nr) {
#pragma unroll
            for (int ii = 0; ii < 4; ++ii) colb[nxt][4 * br + ii] = a[ii][jj];
          }
      }
      if (br == nq && active) {
#pragma unroll
        for (int ii = 0; ii < 4; ++ii)
          if (ii == nr) {
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) xrow[nxt][4 * bc + jj] = x[ii][jj];
          }
      }
    }
    __syncthreads();
  }
  // log-diagonal sum and the first failing pivot, once, by wave 0
  double logsum = 0.0;
  int fail = -1;
  if (tid < 64) {
    const double dj = pivs[tid];
    double lg = (tid < w) ? 0.5 * log(dj) : 0.0;
    const bool bad = (tid < w) && !(dj > 0.0);
    const unsigned long long badmask = __ballot(bad);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) lg += __shfl_xor(lg, off, 64);
    logsum = lg;
    if (badmask) fail = __ffsll((long long)badmask) - 1;
  }

  if (blockIdx.x == 0) {
    double* G = P.G + (long long)z * P.zG;
#pragma unroll
    for (int ii = 0; ii < 4; ++ii)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int r = 4 * br + ii, c = 4 * bc + jj;
        if (r < w && c < w) {
          const long long off = (long long)(c0 + r) + (long long)(c0 + c) * b;
          const bool low = active && r >= c;
          D[off] = low ? a[ii][jj] : 0.0;
          G[off] = low ? x[ii][jj] : 0.0;
        }
      }
    if (tid == 0) {
      P.ldp[(long long)z * P.zLd] = logsum;
      if (fail >= 0) atomicMin(P.info + z, (int32_t)(P.gcol0 + c0 + fail + 1));
    }
    return;
  }

  // panel solve for rows r0..r0+h: L(m, n) = sum_k A(m, k) Linv(n, k)
  const int r0 = c0 + NB * blockIdx.x;
  const int h = min(NB, b - r0);
#pragma unroll
  for (int ii = 0; ii < 4; ++ii)
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int n = 4 * br + ii, k = 4 * bc + jj;  // Linv(n, k), lower
      Xs[k][n] = (active && n >= k) ? x[ii][jj] : 0.0;
    }
  for (int e = tid; e < NB * NB; e += 256) {
    const int m = e & 63, k = e >> 6;
    As[k][m] = (m < h && k < w) ? D[(long long)(r0 + m) + (long long)(c0 + k) * b] : 0.0;
  }
  __syncthreads();
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  v4d acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int kk = 0; kk < NB / 4; ++kk) {
    const int kr = kk * 4 + (lane >> 4);
    const double a0 = As[kr][wm + (lane & 15)];
    const double a1 = As[kr][wm + 16 + (lane & 15)];
    const double b0 = Xs[kr][wn + (lane & 15)];
    const double b1 = Xs[kr][wn + 16 + (lane & 15)];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(b0, a0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(b1, a0, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(b0, a1, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(b1, a1, acc[1][1], 0, 0, 0);
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = wm + bi * 16 + (lane & 15);
        const int n = wn + bj * 16 + (lane >> 4) + 4 * v;
        if (m < h && n < w) D[(long long)(r0 + m) + (long long)(c0 + n) * b] = acc[bi][bj][v];
      }
}

// ---------------------------------------------------------------------------------------------
struct TipArgs {
  double* T; long long zT; int a, ap;    // ap x ap, ld ap; rhs row = row a when ap == a+1
  double* ldp; long long zLd;            // tip log-diagonal sum slot
  int32_t* info; long long gcol0;        // global column of the tip's first column
  double* zsq;                           // per chain |z|^2 (nullable)
  double* ZT; long long zZT;             // a x a (nullable)
  double* xT; long long zXT;             // a (nullable)
};

__global__ __launch_bounds__(64) void tip_kernel(const TipArgs P) {
  constexpr int AMAX = 65;
  __shared__ double L[AMAX][AMAX + 1];
  __shared__ double X[AMAX][AMAX + 1];
  __shared__ double zt[AMAX];
  const int z = blockIdx.x;
  const int a = P.a, ap = P.ap;
  double* T = P.T + (long long)z * P.zT;
  const int tid = threadIdx.x;
  for (int e = tid; e < ap * ap; e += 64) {
    const int r = e % ap, c = e / ap;
    L[r][c] = (r >= c) ? T[r + (long long)c * ap] : 0.0;
  }
  __syncthreads();
  // serial right-looking Cholesky of the leading a x a block (a <= 64, once per sweep)
  int fail = -1;
  double logsum = 0.0;
  for (int j = 0; j < a; ++j) {
    const double d = L[j][j];
    if (!(d > 0.0) && fail < 0) fail = j;
    const double piv = sqrt(d);
    logsum += log(piv);
    __syncthreads();
    if (tid == 0) L[j][j] = piv;
    for (int r = j + 1 + tid; r < ap; r += 64) L[r][j] /= piv;  // includes the rhs row
    __syncthreads();
    const int nr = ap - j - 1, nc = a - j - 1;  // rows include the rhs row
    for (int e = tid; e < nr * nc; e += 64) {
      const int r = j + 1 + e % nr, c = j + 1 + e / nr;
      if (r >= c) L[r][c] -= L[r][j] * L[c][j];
    }
    __syncthreads();
  }
  // X = L_T^-1 (column per thread, forward substitution)
  for (int c = tid; c < a; c += 64) {
    for (int r = 0; r < a; ++r) {
      double s = (r == c) ? 1.0 : 0.0;
      for (int m = c; m < r; ++m) s -= L[r][m] * X[m][c];
      X[r][c] = (r >= c) ? s / L[r][r] : 0.0;
    }
  }
  // z_T = row a of the factor (already L_T^-1 (r_T - v_T))
  if (tid == 0) {
    double zz = 0.0;
    for (int c = 0; c < a; ++c) {
      zt[c] = (ap > a) ? L[a][c] : 0.0;
      zz += zt[c] * zt[c];
    }
    if (P.zsq) P.zsq[z] = (ap > a ? -T[a + (long long)a * ap] : 0.0) + zz;
    P.ldp[(long long)z * P.zLd] = logsum;
    if (fail >= 0) atomicMin(P.info + z, (int32_t)(P.gcol0 + fail + 1));
  }
  __syncthreads();
  for (int e = tid; e < ap * ap; e += 64) {
    const int r = e % ap, c = e / ap;
    if (r < a && c < a) T[r + (long long)c * ap] = (r >= c) ? L[r][c] : 0.0;
    else if (r == a && c < a) T[r + (long long)c * ap] = L[r][c];
  }
  if (P.ZT) {
    double* ZT = P.ZT + (long long)z * P.zZT;
    for (int e = tid; e < a * a; e += 64) {
      const int r = e % a, c = e / a;
      double s = 0.0;
      for (int m = max(r, c); m < a; ++m) s += X[m][r] * X[m][c];
      ZT[r + (long long)c * a] = s;
    }
  }
  if (P.xT) {
    double* xT = P.xT + (long long)z * P.zXT;
    for (int r = tid; r < a; r += 64) {
      double s = 0.0;
      for (int m = r; m < a; ++m) s += X[m][r] * zt[m];
      xT[r] = s;
    }
  }
}

__global__ __launch_bounds__(256) void logdet_reduce_kernel(const double* ldpart, long long zLd,
                                                            int nparts, double* out,
                                                            long long zout) {
  __shared__ double red[256];
  const int z = blockIdx.x;
  const double* p = ldpart + (long long)z * zLd;
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 256) s += p[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[(long long)z * zout] = 2.0 * red[0];
}

}  // namespace

int launch_potrf_panel(double* D, long long zD, double* G, long long zG, double* ldp,
                       long long zLd, int32_t* info, int b, int c0, long long gcol0, int nz,
                       hipStream_t s) {
  PanelArgs P{D, zD, G, zG, ldp, zLd, info, b, c0, gcol0};
  const int rows = (b - c0 + NB - 1) / NB;
  const ProfToken t = prof_begin(s);
  hipLaunchKernelGGL(potrf_panel_kernel, dim3(rows, 1, nz), dim3(256), 0, s, P);
  if (t.valid) {
    // the panel's share of the Cholesky: w^3/3 for the tile, w^2 per row below it
    const double w = (b - c0) < NB ? (b - c0) : NB;
    const double below = (double)(b - c0) - w;
    prof_end(t, s, PK_PANEL, nz * (w * w * w / 3.0 + below * w * w), 0.0);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_tip(double* T, long long zT, int a, int ap, double* ldp, long long zLd, int32_t* info,
               long long gcol0, double* zsq, double* ZT, long long zZT, double* xT,
               long long zXT, int nz, hipStream_t s) {
  if (ap > 65) return -1;
  TipArgs P{T, zT, a, ap, ldp, zLd, info, gcol0, zsq, ZT, zZT, xT, zXT};
  const ProfToken t = prof_begin(s);
  hipLaunchKernelGGL(tip_kernel, dim3(nz), dim3(64), 0, s, P);
  if (t.valid) prof_end(t, s, PK_TIP, nz * (double)a * a * a / 3.0, 0.0);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int bta_logdet_reduce(const double* ldpart, long long zLd, int nparts, double* out, long long zout,
                      int nz, hipStream_t s) {
  hipLaunchKernelGGL(logdet_reduce_kernel, dim3(nz), dim3(256), 0, s, ldpart, zLd, nparts, out,
                     zout);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace adelia
