// Small HBM-bound helper kernels: fills, strided block copies, and the matrix-vector products of
// the triangular solves (Sec. III-A-2, Eqs. 3-5).  Reductions use a fixed order (no atomics)
// so that repeated runs are bitwise identical.
#include "common.h"
#include "launchers.h"
#include "profile.h"
#include <climits>

namespace adelia {

namespace {

__global__ void fill_kernel(double* p, long long n, double v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void fill_i32_kernel(int32_t* p, long long n, int32_t v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

// dst(r, c) = src(r, c) for r < rows, c < cols; chain z = blockIdx.z
__global__ void copy2d_kernel(const double* src, long long lds, long long zs_src, double* dst,
                              long long ldd, long long zs_dst, int rows, int cols) {
  const int z = blockIdx.z;
  const long long total = (long long)rows * cols;
  const double* s = src + (long long)z * zs_src;
  double* d = dst + (long long)z * zs_dst;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long r = e % rows, c = e / rows;
    d[r + c * ldd] = s[r + c * lds];
  }
}

// zero the strict upper triangle of nblk b x b blocks (block stride `bs`, ld) per chain
__global__ void zero_upper_kernel(double* p, int b, long long ld, long long bs, int nblk,
                                  long long zs) {
  const int z = blockIdx.z;
  const int blk = blockIdx.y;
  double* q = p + (long long)z * zs + (long long)blk * bs;
  const long long total = (long long)b * b;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long r = e % b, c = e / b;
    if (r < c) q[r + c * ld] = 0.0;
  }
}

// One wavefront per output element m: y(m) = beta*y0(m) + alpha*sum_k A(k,m) x(k)
//                                             + alpha2*sum_c A2(c,m) x2(c)
__global__ __launch_bounds__(256) void gemv_t_kernel(const GemvT g) {
  const int z = blockIdx.z;
  if (g.zn && g.step >= g.zn[(long long)z * g.zn_stride]) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = blockIdx.x * 4 + wave;
  if (m >= g.M) return;
  double s = 0.0;
  if (g.A && g.alpha != 0.0) {
    const double* col = g.A + (long long)z * g.zA + (long long)m * g.ld;
    const double* x = g.x + (long long)z * g.zx;
    const int k0 = g.lowerA ? m : 0;
    double t = 0.0;
    for (int k = k0 + lane; k < g.K; k += 64) t += col[k] * x[(long long)k * g.incx];
    s += g.alpha * t;
  }
  double s2 = 0.0;
  if (g.A2 && g.r2 > 0 && lane < g.r2) {
    const double* a2 = g.A2 + (long long)z * g.zA2 + (long long)m * g.ld2;
    s2 = a2[lane] * g.x2[(long long)z * g.zx2 + lane];
  }
  s += g.alpha2 * s2;
  // fixed-order butterfly reduction across the wavefront
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) {
    double v = s;
    if (g.beta != 0.0) v += g.beta * g.y0[(long long)z * g.zy0 + (long long)m * g.incy0];
    g.y[(long long)z * g.zy + (long long)m * g.incy] = v;
  }
}

// y(m) = beta*y0(m) + alpha * sum_k A(m,k) x(k), k <= m if lowerA; 64 rows per workgroup,
// the four wavefronts split k and combine in LDS in a fixed order.
struct GemvN {
  const double* A; long long ld; long long zA;
  const double* x; long long zx; long long incx;
  const double* y0; long long zy0; long long incy0;
  double* y; long long zy; long long incy;
  int M, K, lowerA; double alpha, beta;
};

__global__ __launch_bounds__(256) void gemv_n_kernel(const GemvN g) {
  __shared__ double part[4][64];
  const int z = blockIdx.z;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = blockIdx.x * 64 + lane;
  double t = 0.0;
  if (m < g.M) {
    const double* A = g.A + (long long)z * g.zA;
    const double* x = g.x + (long long)z * g.zx;
    const int kend = g.lowerA ? min(g.K, m + 1) : g.K;
    for (int k = wave; k < kend; k += 4) t += A[m + (long long)k * g.ld] * x[(long long)k * g.incx];
  }
  part[wave][lane] = t;
  __syncthreads();
  if (wave == 0 && m < g.M) {
    double s = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
    double v = g.alpha * s;
    if (g.beta != 0.0) v += g.beta * g.y0[(long long)z * g.zy0 + (long long)m * g.incy0];
    g.y[(long long)z * g.zy + (long long)m * g.incy] = v;
  }
}

// Small dense triangular solve with one thread per chain (tip systems, a <= 64):
//   trans == 0: solve L v = v  (forward), trans == 1: solve L^T v = v (backward).
__global__ void tri_small_kernel(const double* L, long long ld, long long zL, double* v,
                                 long long zv, int a, int trans, int nz) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= nz) return;
  const double* l = L + (long long)z * zL;
  double* x = v + (long long)z * zv;
  if (!trans) {
    for (int r = 0; r < a; ++r) {
      double s = x[r];
      for (int m = 0; m < r; ++m) s -= l[r + m * ld] * x[m];
      x[r] = s / l[r + r * ld];
    }
  } else {
    for (int r = a - 1; r >= 0; --r) {
      double s = x[r];
      for (int m = r + 1; m < a; ++m) s -= l[m + r * ld] * x[m];
      x[r] = s / l[r + r * ld];
    }
  }
}

// per-block sum of log(L_jj) over the diagonal of nblk b x b blocks -> part[blk]
__global__ __launch_bounds__(256) void logdiag_kernel(const double* L, int b, long long ld,
                                                      long long bs, double* part, long long zL,
                                                      long long zp) {
  __shared__ double red[256];
  const int z = blockIdx.z, blk = blockIdx.x;
  const double* q = L + (long long)z * zL + (long long)blk * bs;
  double s = 0.0;
  for (int j = threadIdx.x; j < b; j += 256) s += log(q[j + (long long)j * ld]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(long long)z * zp + blk] = red[0];
}

inline unsigned grid_for(long long n) {
  long long g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (unsigned)g;
}

}  // namespace

// C(r, n) = alpha * (sum_k A1(r, k) B1(k, n) + sum_k A2(r, k) B2(k, n)) + beta * C(r, n) for the
// m <= kSkinnyRows rows of a short, wide product (column-major operands; A2/B2 may be absent).
// Each wavefront takes kSkinnyCols columns; its lanes walk K (coalesced reads of B's columns),
// each lane reads the m values of A at its k once for all its columns, and the 64 partial sums
// are combined by a fixed-order reduce-scatter butterfly that leaves sum i on lane i.
__global__ __launch_bounds__(256) void skinny_kernel(const Skinny g) {
  const int z = blockIdx.z;
  if (z_idle(g.zn, g.step, g.zdiv, z)) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n0 = (blockIdx.x * 4 + wave) * kSkinnyCols;
  if (n0 >= g.N) return;
  double v[kSkinnyRows * kSkinnyCols];
#pragma unroll
  for (int i = 0; i < kSkinnyRows * kSkinnyCols; ++i) v[i] = 0.0;
  // lower: B(k, n) = 0 for k < n, so the walk starts at the wave's first column and each column
  // masks the rows above its own
  auto part = [&](const double* A, long long lda, const double* B, long long ldb, int K,
                  bool lower) {
    for (int k = (lower ? n0 : 0) + lane; k < K; k += 64) {
      double av[kSkinnyRows];
#pragma unroll
      for (int r = 0; r < kSkinnyRows; ++r) av[r] = r < g.m ? A[r + (long long)k * lda] : 0.0;
#pragma unroll
      for (int j = 0; j < kSkinnyCols; ++j) {
        const double bl = B[k + (long long)min(n0 + j, g.N - 1) * ldb];
        const double bv = (lower && k < n0 + j) ? 0.0 : bl;
#pragma unroll
        for (int r = 0; r < kSkinnyRows; ++r) v[r * kSkinnyCols + j] = fma(av[r], bv, v[r * kSkinnyCols + j]);
      }
    }
  };
  part(g.A1 + (long long)z * g.zA1, g.lda1, g.B1 + (long long)z * g.zB1, g.ldb1, g.K1,
       g.lowerB != 0);
  if (g.A2 && g.K2 > 0)
    part(g.A2 + (long long)z * g.zA2, g.lda2, g.B2 + (long long)z * g.zB2, g.ldb2, g.K2, false);
  // reduce-scatter: at offset o a lane keeps half of its current values (the upper half if bit
  // o of its lane id is set) and adds the partner's copy of that half
#pragma unroll
  for (int o = 32, cnt = 64; o >= 1; o >>= 1, cnt >>= 1) {
    const bool up = (lane & o) != 0;
#pragma unroll
    for (int i = 0; i < cnt / 2; ++i) {
      const double send = up ? v[i] : v[i + cnt / 2];
      const double keep = up ? v[i + cnt / 2] : v[i];
      v[i] = keep + __shfl_xor(send, o, 64);
    }
  }
  const int r = lane / kSkinnyCols, n = n0 + lane % kSkinnyCols;
  if (r < g.m && n < g.N) {
    double* c = g.C + (long long)z * g.zC + r + (long long)n * g.ldc;
    *c = g.alpha * v[0] + (g.beta != 0.0 ? g.beta * *c : 0.0);
  }
}

int launch_fill(double* p, long long n, double v, hipStream_t s) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_fill_i32(int32_t* p, long long n, int32_t v, hipStream_t s) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_copy2d(const double* src, long long lds, long long zs_src, double* dst, long long ldd,
                  long long zs_dst, int rows, int cols, int nz, hipStream_t s) {
  if (rows <= 0 || cols <= 0 || nz <= 0) return 0;
  hipLaunchKernelGGL(copy2d_kernel, dim3(grid_for((long long)rows * cols), 1, nz), dim3(256), 0,
                     s, src, lds, zs_src, dst, ldd, zs_dst, rows, cols);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_zero_upper(double* p, int b, long long ld, long long blockstride, int nblk,
                      long long zs, int nz, hipStream_t s) {
  if (b <= 1 || nblk <= 0 || nz <= 0) return 0;
  hipLaunchKernelGGL(zero_upper_kernel, dim3(grid_for((long long)b * b), nblk, nz), dim3(256), 0,
                     s, p, b, ld, blockstride, nblk, zs);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_gemv_t(const GemvT& g, int nz, hipStream_t s) {
  if (g.M <= 0 || nz <= 0) return 0;
  if (g.r2 > 64) return -1;
  const ProfToken t = prof_begin(s);
  hipLaunchKernelGGL(gemv_t_kernel, dim3((g.M + 3) / 4, 1, nz), dim3(256), 0, s, g);
  if (t.valid) {
    const double elems = g.A ? (g.lowerA ? 0.5 * g.M * (g.M + 1.0) : (double)g.M * g.K) : 0.0;
    prof_end(t, s, PK_GEMV, nz * 2.0 * elems, nz * 8.0 * (elems + (double)g.r2 * g.M + 2.0 * g.M));
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_gemv_n(const double* A, long long ld, long long zA, const double* x, long long zx,
                  long long incx, const double* y0, long long zy0, long long incy0, double* y,
                  long long zy, long long incy, int M, int K, int lowerA, double alpha,
                  double beta, int nz, hipStream_t s) {
  if (M <= 0 || nz <= 0) return 0;
  GemvN g{A, ld, zA, x, zx, incx, y0, zy0, incy0, y, zy, incy, M, K, lowerA, alpha, beta};
  hipLaunchKernelGGL(gemv_n_kernel, dim3((M + 63) / 64, 1, nz), dim3(256), 0, s, g);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_tri_small(const double* L, long long ld, long long zL, double* v, long long zv, int a,
                     int trans, int nz, hipStream_t s) {
  if (a <= 0 || nz <= 0) return 0;
  hipLaunchKernelGGL(tri_small_kernel, dim3((nz + 63) / 64), dim3(64), 0, s, L, ld, zL, v, zv, a,
                     trans, nz);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_logdiag(const double* L, int b, long long ld, long long bs, int nblk, double* part,
                   long long zL, long long zp, int nz, hipStream_t s) {
  if (nblk <= 0 || nz <= 0) return 0;
  hipLaunchKernelGGL(logdiag_kernel, dim3(nblk, 1, nz), dim3(256), 0, s, L, b, ld, bs, part, zL,
                     zp);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace adelia

namespace adelia {
namespace {
__global__ void fill_strided_kernel(double* p, long long stride, int count, double v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[(long long)i * stride] = v;
}
}  // namespace
int launch_fill_strided(double* p, long long stride, int count, double v, hipStream_t s) {
  if (count <= 0) return 0;
  hipLaunchKernelGGL(fill_strided_kernel, dim3((count + 255) / 256), dim3(256), 0, s, p, stride,
                     count, v);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
int launch_skinny(const Skinny& g, int nz, hipStream_t s) {
  if (g.m < 1 || g.m > kSkinnyRows || g.N < 0 || g.K1 < 0 || g.K2 < 0 || nz < 1 || nz > 65535)
    return -1;
  if (g.N == 0) return 0;
  const ProfToken t = prof_begin(s);
  hipLaunchKernelGGL(skinny_kernel, dim3((g.N + 4 * kSkinnyCols - 1) / (4 * kSkinnyCols), 1, nz),
                     dim3(256), 0, s, g);
  if (t.valid) {
    // products taking part: all of the second pair; of the first, those on or below B1's
    // diagonal when it is lower triangular
    const double k1 = g.lowerB ? (double)g.N * g.K1 - 0.5 * (double)g.N * (g.N - 1)
                               : (double)g.N * g.K1;
    const double kk = k1 + (double)g.N * g.K2;
    prof_end(t, s, PK_GEMV, nz * 2.0 * g.m * kk,
             nz * 8.0 * (kk + (double)g.m * (g.K1 + g.K2) + g.m * g.N));
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace adelia
