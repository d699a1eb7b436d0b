// Diagonal-block Cholesky pieces of the BTA sweep (Sec. III-A-1, Alg. 1, the chol() steps).
//
// The panel step of the blocked Cholesky of a diagonal block is in panel.hip; the trailing
// update between panels is a GEMM launch (gemm.hip).
//
// tip_kernel: factors the a x a arrowhead tip after the sweep, finishes the forward solve
// (z_T), and forms Z_T = L_T^-T L_T^-1 and x_T = L_T^-T z_T for the backward pass.
#include "common.h"
#include "profile.h"
#include <cmath>

namespace adelia {

namespace {

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
