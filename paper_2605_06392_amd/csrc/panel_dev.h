// Panel step of the blocked Cholesky of a diagonal block (Sec. III-A-1, Alg. 1, chol()).
//
// The 64 x 64 diagonal tile of panel k is factored, together with its inverse, as two 32 x 32
// leaves, each two 16 x 16 leaves eliminated by ONE wavefront four columns per step in the
// matrix cores' accumulator layout (each step's rank-4 updates of the leaf and of its inverse
// are one 16 x 16 x 4 product each; a single wave needs no workgroup barrier because its LDS
// operations complete in program order), and the off-diagonal solve L21 = A21 X11^T, the
// update A22 -= L21 L21^T and the inverse merge X21 = -X22 L21 X11 run on the matrix cores
// across the four waves.  Workgroup x > 0 also solves its 64-row tile of the panel as
// A_jk L_kk^-T.
//
// The leaves are serial, so the other three waves work beside them: with the look-ahead
// update (the previous panel's rank-64 contribution to this panel's columns, applied here
// instead of by the trailing update) only the first leaf's 32 x 32 block of it precedes the
// first leaf; the rest of the diagonal tile's update and the updated row tile are formed
// during the first leaf, and the row tile's first 32 columns, R1 = W1 X11^T, together with
// W2 -= R1 L21^T, during the second.  What is left after the leaves is R2 = W2 X22^T.
//
// Every workgroup reads the unfactored diagonal tile, so L_kk may only be written back once
// all of them have loaded it: each workgroup bumps a per-chain counter after its load, and the
// one that sees the count complete stores L_kk (all workgroups compute bit-identical tiles) and
// resets the counter for the next launch.  L_kk^-1, the log-diagonal sum and the pivot check,
// which no workgroup of the launch reads, are formed and stored by workgroup 0 (it owns no row
// tile).  No workgroup ever waits on another.
#pragma once
#include "common.h"
#include <cmath>

namespace adelia {
namespace panel_dev {

constexpr int NB = kPanel;  // 64
constexpr int HB = NB / 2;  // 32
constexpr int LP = NB + 1;  // LDS pitch of the square tiles

struct PanelArgs {
  double* D; long long zD;
  double* G; long long zG;
  double* ldp; long long zLd;
  int32_t* info;
  int32_t* cnt;  // per chain, zero between launches
  const int32_t* zn;  // per chain block count (uneven batch) or nullptr
  int step;
  int b, c0;
  long long gcol0;
  // rows below the block solved with the same panel (Alg. 1: [B_i; C_i] against L_Di^T):
  // mT rows of T (ld ldT, chain stride zT), nullptr when none
  double* T; long long zT;
  int ldT, mT;
  // apply the previous panel's rank-64 update to this panel's columns first (the trailing
  // update of the remaining columns then runs beside the next panels)
  int upd;
  // if not null (and upd): workgroup 0 also stores V = L_kk^-1 Q (64 x 64, column-major, chain
  // stride zV), Q the previous panel's columns on the diagonal rows, so that rows solved
  // elsewhere get R = A L_kk^-T - P V^T without the updated diagonal tile
  double* V; long long zV;
};

// Orders the LDS traffic of one wavefront: the LDS unit serves a wave's operations in issue
// order, so a compiler-level barrier is all a single wave needs between producer and consumer.
__device__ __forceinline__ void wave_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 1/sqrt(d) from the hardware estimate refined by two Newton steps (each squares the relative
// error), and sqrt(d) = d / sqrt(d).  A non-positive d gives a NaN or an infinity, which the
// caller reports through the pivot check.
__device__ __forceinline__ void pivot(double d, double& pv, double& invs) {
  double r = __builtin_amdgcn_rsq(d);
  const double h = 0.5 * d;
  r = r * fma(-h * r, r, 1.5);
  r = r * fma(-h * r, r, 1.5);
  invs = r;
  pv = d * r;
}

constexpr int QB = 16;  // edge of the serially eliminated leaves

// A double from lane `src` of the wavefront (src a compile-time constant: uniform).
__device__ __forceinline__ double lane_value(double v, int src) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, src);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), src);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// One step of the 16 x 16 leaf: columns j0 = 4 JQ .. j0 + 3.  The wavefront holds the leaf A
// (being overwritten by L) and X^T (X becoming L^-1) in the accumulator layout of the matrix
// cores: lane (m, c) = (lane % 16, lane / 16) holds column c + 4v of row m, v = 0..3.  So the
// column block of this step is s[JQ], element (m, j0 + c) on lane (m, c).  Every lane factors
// the 4 x 4 pivot block itself (read from the lanes holding it; the result is the same on
// every lane) into L_p and M = L_p^-1; then lane (m, c) forms L(m, j0 + c) = sum_c' A(m, j0 + c')
// M(c, c') and the scaled pivot row X_new(j0 + c, m) = sum_c' M(c, c') X(j0 + c', m) from the
// three other lanes of its row, and the rank-4 updates of the trailing part of A and of the rows
// of X below the block are each one 16 x 16 x 4 product with those values as its operands.
template <int JQ>
__device__ __forceinline__ void leaf_step(v4d& s, v4d& xt, double* piv, int o, int m, int c,
                                          int lane) {
  constexpr int j0 = 4 * JQ;
  // the pivot block (lower part), from the lanes holding it
  double P[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int q = 0; q <= r; ++q) P[r][q] = lane_value(s[JQ], (j0 + r) + 16 * q);
  // row m of the block column and rows j0.. of X at column m, from the lanes of row m
  double a[4], xs[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    a[q] = __shfl(s[JQ], m + 16 * q, 64);
    xs[q] = __shfl(xt[JQ], m + 16 * q, 64);
  }
  // L_p (pivots d_r, reciprocal square roots r_r) and M = L_p^-1
  double d0, d1, d2, d3, p0, p1, p2, p3, r0, r1, r2, r3;
  d0 = P[0][0];
  pivot(d0, p0, r0);
  const double l10 = P[1][0] * r0, l20 = P[2][0] * r0, l30 = P[3][0] * r0;
  d1 = fma(-l10, l10, P[1][1]);
  pivot(d1, p1, r1);
  const double l21 = fma(-l20, l10, P[2][1]) * r1, l31 = fma(-l30, l10, P[3][1]) * r1;
  d2 = fma(-l21, l21, fma(-l20, l20, P[2][2]));
  pivot(d2, p2, r2);
  const double l32 = fma(-l31, l21, fma(-l30, l20, P[3][2])) * r2;
  d3 = fma(-l32, l32, fma(-l31, l31, fma(-l30, l30, P[3][3])));
  pivot(d3, p3, r3);
  if (lane == 0) {
    piv[o + j0] = d0;
    piv[o + j0 + 1] = d1;
    piv[o + j0 + 2] = d2;
    piv[o + j0 + 3] = d3;
  }
  const double M10 = -r1 * (l10 * r0);
  const double M21 = -r2 * (l21 * r1);
  const double M20 = -r2 * fma(l21, M10, l20 * r0);
  const double M32 = -r3 * (l32 * r2);
  const double M31 = -r3 * fma(l32, M21, l31 * r1);
  const double M30 = -r3 * fma(l32, M20, fma(l31, M10, l30 * r0));
  // row c of M (zero right of the diagonal)
  const double mc0 = c == 0 ? r0 : (c == 1 ? M10 : (c == 2 ? M20 : M30));
  const double mc1 = c == 0 ? 0.0 : (c == 1 ? r1 : (c == 2 ? M21 : M31));
  const double mc2 = c <= 1 ? 0.0 : (c == 2 ? r2 : M32);
  const double mc3 = c <= 2 ? 0.0 : r3;
  double ell = fma(a[3], mc3, fma(a[2], mc2, fma(a[1], mc1, a[0] * mc0)));
  const double xn = fma(mc3, xs[3], fma(mc2, xs[2], fma(mc1, xs[1], mc0 * xs[0])));
  // L(m, j0 + c) lives on or below the diagonal; the rows below the block update X
  ell = m >= j0 + c ? ell : 0.0;
  const double ellb = m >= j0 + 4 ? ell : 0.0;
  s = __builtin_amdgcn_mfma_f64_16x16x4f64(ell, -ell, s, 0, 0, 0);
  xt = __builtin_amdgcn_mfma_f64_16x16x4f64(ellb, -xn, xt, 0, 0, 0);
  s[JQ] = ell;
  xt[JQ] = xn;
}

// Factor the 16 x 16 leaf at (o, o) of S (lower triangle, already updated) with one wavefront.
// On exit S holds L (lower, zeros above) and X holds L^-1 on that leaf; piv[o + j] = pivot^2.
__device__ void leaf16(double (*S)[LP], double (*X)[LP], double* piv, int o) {
  const int lane = threadIdx.x & 63;
  const int m = lane & 15, c = lane >> 4;
  v4d s, xt;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int n = c + 4 * v;
    const double val = S[o + m][o + n];
    s[v] = m >= n ? val : 0.0;
    xt[v] = m == n ? 1.0 : 0.0;
  }
  leaf_step<0>(s, xt, piv, o, m, c, lane);
  leaf_step<1>(s, xt, piv, o, m, c, lane);
  leaf_step<2>(s, xt, piv, o, m, c, lane);
  leaf_step<3>(s, xt, piv, o, m, c, lane);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int n = c + 4 * v;
    S[o + m][o + n] = m >= n ? s[v] : 0.0;  // L(m, n)
    X[o + n][o + m] = n >= m ? xt[v] : 0.0;  // X(n, m) from X^T(m, n)
  }
  wave_order();
}

// One 16 x 16 fragment C = sum_k A(m, k) B(k, n), k < K (K a multiple of 4), computed by the
// calling wavefront at (fm, fn): lane holds C(fm + lane%16, fn + lane/16 + 4v).
template <class FA, class FB>
__device__ __forceinline__ v4d frag16(FA A, FB B, int fm, int fn, int K) {
  const int lane = threadIdx.x & 63;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  for (int kk = 0; kk < K / 4; ++kk) {
    const int k = kk * 4 + (lane >> 4);
    const double av = A(fm + (lane & 15), k);
    const double bv = B(k, fn + (lane & 15));
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(bv, av, acc, 0, 0, 0);
  }
  return acc;
}

// Factor the 32 x 32 block at (o, o) of S, with its inverse in X, by one wavefront: two serial
// 16 x 16 leaves, the coupling L21 = A21 X11^T, the update A22 -= L21 L21^T and the inverse
// merge X21 = -X22 (L21 X11) on the matrix cores.  The wave orders its own LDS traffic, so no
// workgroup barrier is needed; every fragment is read completely before it is overwritten.
__device__ void leaf32(double (*S)[LP], double (*X)[LP], double* piv, int o) {
  const int lane = threadIdx.x & 63;
  const int m = lane & 15, n0 = lane >> 4;
  const int h = o + QB;
  leaf16(S, X, piv, o);
  v4d t = frag16([&](int r, int k) { return S[h + r][o + k]; },
                 [&](int k, int c) { return X[o + c][o + k]; }, 0, 0, QB);
#pragma unroll
  for (int v = 0; v < 4; ++v) S[h + m][o + n0 + 4 * v] = t[v];
  wave_order();
  t = frag16([&](int r, int k) { return S[h + r][o + k]; },
             [&](int k, int c) { return S[h + c][o + k]; }, 0, 0, QB);
#pragma unroll
  for (int v = 0; v < 4; ++v) S[h + m][h + n0 + 4 * v] -= t[v];
  wave_order();
  leaf16(S, X, piv, h);
  t = frag16([&](int r, int k) { return S[h + r][o + k]; },
             [&](int k, int c) { return X[o + k][o + c]; }, 0, 0, QB);
#pragma unroll
  for (int v = 0; v < 4; ++v) X[h + m][o + n0 + 4 * v] = t[v];
  wave_order();
  t = frag16([&](int r, int k) { return X[h + r][h + k]; },
             [&](int k, int c) { return X[h + k][o + c]; }, 0, 0, QB);
#pragma unroll
  for (int v = 0; v < 4; ++v) X[h + m][o + n0 + 4 * v] = -t[v];
  wave_order();
}

// One 16 x 16 fragment of a 32 x 32 product C = sum_k A(m, k) B(k, n), k < 32, computed by the
// calling wavefront: lane holds C(fm + lane%16, fn + lane/16 + 4v).
template <class FA, class FB>
__device__ __forceinline__ v4d frag32(FA A, FB B, int fm, int fn) {
  return frag16(A, B, fm, fn, HB);
}

// acc[j] += sum_{k < K} A[am + m][ak + k] B[16 j + n][bk + k] for one 16-row strip (m < 16) and
// the column fragments j < NJ: lane holds (am + lane%16, 16 j + lane/16 + 4v).
template <int NJ, int K>
__device__ __forceinline__ void strip_abt(const double (*A)[LP], int am, int ak,
                                          const double (*B)[LP], int bk, int lane,
                                          v4d (&acc)[NJ]) {
  const int lm = lane & 15, lk = lane >> 4;
#pragma unroll 4
  for (int kk = 0; kk < K / 4; ++kk) {
    const double av = A[am + lm][ak + 4 * kk + lk];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const double bv = B[16 * j + lm][bk + 4 * kk + lk];
      acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv, av, acc[j], 0, 0, 0);
    }
  }
}

// LDS of one panel workgroup (134 KB: one workgroup per CU).
struct PanelSmem {
  double S[NB][LP];  // diagonal tile, factored in place into L_kk
  double X[NB][LP];  // L_kk^-1
  double Q[NB][LP];  // previous panel on the diagonal tile's rows (with the update)
  double W[NB][LP];  // previous panel on this tile's rows, then the updated row tile
  double piv[NB];
  int writer;
};

// One workgroup of a panel launch: workgroup bx of nbx of chain z.
__device__ __forceinline__ void panel_body(const PanelArgs& P, int bx, int nbx, PanelSmem& sm,
                                           int z) {
  double (*S)[LP] = sm.S;
  double (*X)[LP] = sm.X;
  double (*Q)[LP] = sm.Q;
  double (*W)[LP] = sm.W;
  double* piv = sm.piv;
  int& writer = sm.writer;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lm = lane & 15, lk = lane >> 4;
  if (P.zn && P.step >= P.zn[z]) return;  // chain z has no block at this step
  const int b = P.b, c0 = P.c0;
  const int w = min(NB, b - c0);
  double* D = P.D + (long long)z * P.zD;
  // workgroup x > 0 owns a 64-row tile: first the block's own rows below the diagonal tile,
  // then the rows of T
  const int nd = (b - c0 + NB - 1) / NB;  // diagonal tile + block rows
  const bool rows = bx > 0;
  const bool tall = (int)bx >= nd;
  double* R = tall ? P.T + (long long)z * P.zT : D;
  const long long ldR = tall ? P.ldT : b;
  const int r0 = tall ? NB * ((int)bx - nd) : c0 + NB * bx;
  const int h = rows ? min(NB, (tall ? P.mT : b) - r0) : 1;
  const bool upd = P.upd && c0 >= NB;
  // 16-row strips of the row tile kept by waves 1..3 while wave 0 factors the leaves
  const int s0 = wave == 1 ? 0 : wave, ns = wave == 0 ? 0 : (wave == 1 ? 2 : 1);
  // Every global read is issued here, back to back (addresses clamped into the tiles, values
  // masked on use): the diagonal tile, the previous panel's columns on it and on this tile's
  // rows, and the row tile itself, which waves 1..3 load in the matrix-core accumulator layout.
  double dv[NB * NB / 256], qv[NB * NB / 256], pv[NB * NB / 256], rt[2][4][4];
#pragma unroll
  for (int i = 0; i < NB * NB / 256; ++i) {
    const int e = tid + 256 * i, r = e & 63, c = e >> 6;
    dv[i] = D[(long long)(c0 + min(r, w - 1)) + (long long)(c0 + min(c, w - 1)) * b];
  }
  if (upd) {
#pragma unroll
    for (int i = 0; i < NB * NB / 256; ++i) {
      const int e = tid + 256 * i, r = e & 63, k = e >> 6;
      qv[i] = D[(long long)(c0 + min(r, w - 1)) + (long long)(c0 - NB + k) * b];
    }
    if (rows) {
#pragma unroll
      for (int i = 0; i < NB * NB / 256; ++i) {
        const int e = tid + 256 * i, m = e & 63, k = e >> 6;
        pv[i] = R[(long long)(r0 + min(m, h - 1)) + (long long)(c0 - NB + k) * ldR];
      }
    }
  }
  if (rows && wave > 0) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      if (s >= ns) break;
      const int m = min(16 * (s0 + s) + lm, h - 1);
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          rt[s][j][v] = R[(long long)(r0 + m) + (long long)(c0 + min(16 * j + lk + 4 * v, w - 1)) * ldR];
    }
  }
  // diagonal tile (lower) with identity padding past w
#pragma unroll
  for (int i = 0; i < NB * NB / 256; ++i) {
    const int e = tid + 256 * i, r = e & 63, c = e >> 6;
    const double v = (r < w && c < w) ? dv[i] : (r == c ? 1.0 : 0.0);
    S[r][c] = (r >= c) ? v : 0.0;
    X[r][c] = 0.0;
    if (upd) {
      Q[r][c] = (r < w) ? qv[i] : 0.0;
      if (rows) W[r][c] = (r < h) ? pv[i] : 0.0;
    }
  }
  __syncthreads();  // this workgroup's reads of the diagonal tile have completed
  if (tid == 0) {
    const int seen = atomicAdd(P.cnt + z, 1);
    const bool last = seen == (int)nbx - 1;
    if (last) atomicExch(P.cnt + z, 0);
    writer = last ? 1 : 0;
  }
  if (upd) {
    // rank-64 update of the first leaf's block: S -= Q Q^T on fragments (0,0), (16,0), (16,16)
    // (the strictly upper part of S is never read)
    if (wave < 3) {
      const int fm = wave == 0 ? 0 : 16, fn = wave == 2 ? 16 : 0;
      const v4d t = frag16([&](int m, int k) { return Q[m][k]; },
                           [&](int k, int n) { return Q[n][k]; }, fm, fn, NB);
#pragma unroll
      for (int v = 0; v < 4; ++v) S[fm + lm][fn + lk + 4 * v] -= t[v];
    }
    __syncthreads();
  }
  if (wave == 0) {
    leaf32(S, X, piv, 0);
  } else {
    // beside the first leaf (which touches rows 0..31 of S and X only): the rest of the
    // diagonal tile's update, rows 32..63 (waves 2 and 3), and the updated row tile
    // W = A - P Q^T, strip by strip, each strip read and rewritten by its own wave
    if (upd && wave >= 2) {
      const int fm = 32 + 16 * (wave - 2);
      for (int fn = 0; fn <= fm; fn += 16) {
        const v4d t = frag16([&](int m, int k) { return Q[m][k]; },
                             [&](int k, int n) { return Q[n][k]; }, fm, fn, NB);
#pragma unroll
        for (int v = 0; v < 4; ++v) S[fm + lm][fn + lk + 4 * v] -= t[v];
      }
    }
    if (rows) {
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        if (s >= ns) break;
        const int mi = s0 + s, m = 16 * mi + lm;
        v4d acc[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            acc[j][v] = (m < h && 16 * j + lk + 4 * v < w) ? -rt[s][j][v] : 0.0;
        if (upd) strip_abt<4, NB>(W, 16 * mi, 0, Q, 0, lane, acc);
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) W[m][16 * j + lk + 4 * v] = -acc[j][v];
      }
    }
  }
  __syncthreads();
  const int fm = (wave & 1) * 16, fn = (wave >> 1) * 16;
  // L21 = A21 X11^T
  v4d t = frag32([&](int m, int k) { return S[HB + m][k]; },
                 [&](int k, int n) { return X[n][k]; }, fm, fn);
  __syncthreads();
#pragma unroll
  for (int v = 0; v < 4; ++v) S[HB + fm + lm][fn + lk + 4 * v] = t[v];
  __syncthreads();
  // A22 -= L21 L21^T (each wave owns its fragment; the strictly upper one is never read)
  t = frag32([&](int m, int k) { return S[HB + m][k]; },
             [&](int k, int n) { return S[HB + n][k]; }, fm, fn);
#pragma unroll
  for (int v = 0; v < 4; ++v) S[HB + fm + lm][HB + fn + lk + 4 * v] -= t[v];
  __syncthreads();
  if (wave == 0) {
    leaf32(S, X, piv, HB);
  } else if (rows) {
    // beside the second leaf (columns 32..63 of S and X): the row tile's first half
    // R1 = W1 X11^T, stored at once, and W2 -= R1 L21^T, so that R2 = W2 X22^T is all that
    // waits for the leaf.  R1's accumulator layout is the A-operand layout of the second product.
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      if (s >= ns) break;
      const int mi = s0 + s, m = 16 * mi + lm;
      v4d r1[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
      strip_abt<2, HB>(W, 16 * mi, 0, X, 0, lane, r1);
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int n = 16 * j + lk + 4 * v;
          if (m < h && n < w) R[(long long)(r0 + m) + (long long)(c0 + n) * ldR] = r1[j][v];
        }
      v4d u[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
#pragma unroll
      for (int kk = 0; kk < HB / 4; ++kk) {
        const double av = r1[kk >> 2][kk & 3];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const double bv = S[HB + 16 * j + lm][4 * kk + lk];
          u[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv, av, u[j], 0, 0, 0);
        }
      }
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) W[m][HB + 16 * j + lk + 4 * v] -= u[j][v];
    }
  }
  __syncthreads();

  // L_kk is stored by the writer (the last workgroup to have loaded the unfactored tile); the
  // inverse, the log-diagonal and the pivot check, which no workgroup of this launch reads, by
  // workgroup 0, which owns no row tile and would otherwise idle while the others solve theirs
  // (when it is also the writer it does both).  Thread (r, q) = (tid % 64, tid / 64) stores the
  // column entries (r, q + 4 i).
  const int wr = tid & (NB - 1), wq = tid >> 6;
  if (writer) {
#pragma unroll 4
    for (int cc = wq; cc < w; cc += 4)
      if (wr < w) D[(long long)(c0 + wr) + (long long)(c0 + cc) * b] = (wr >= cc) ? S[wr][cc] : 0.0;
  }
  if (bx == 0) {
    if (wave == 0) {
      const double dj = piv[lane];
      double lg = (lane < w) ? 0.5 * log(dj) : 0.0;
      const bool bad = (lane < w) && !(dj > 0.0);
      const unsigned long long badmask = __ballot(bad);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) lg += __shfl_xor(lg, off, 64);
      if (lane == 0) {
        P.ldp[(long long)z * P.zLd] = lg;
        if (badmask) atomicMin(P.info + z, (int32_t)(P.gcol0 + c0 + __ffsll((long long)badmask) - 1 + 1));
      }
    }
    // X21 = -X22 (L21 X11), needed only for the stored inverse
    t = frag32([&](int m, int k) { return S[HB + m][k]; },
               [&](int k, int n) { return X[k][n]; }, fm, fn);
#pragma unroll
    for (int v = 0; v < 4; ++v) X[HB + fm + lm][fn + lk + 4 * v] = t[v];
    __syncthreads();
    t = frag32([&](int m, int k) { return X[HB + m][HB + k]; },
               [&](int k, int n) { return X[HB + k][n]; }, fm, fn);
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) X[HB + fm + lm][fn + lk + 4 * v] = -t[v];
    __syncthreads();
    double* G = P.G + (long long)z * P.zG;
#pragma unroll 4
    for (int cc = wq; cc < w; cc += 4)
      if (wr < w) G[(long long)(c0 + wr) + (long long)(c0 + cc) * b] = (wr >= cc) ? X[wr][cc] : 0.0;
    if (P.V && upd) {
      // V = X Q: wave q takes rows 16q..16q+15 (X is zero past w and above the diagonal)
      double* V = P.V + (long long)z * P.zV;
#pragma unroll
      for (int fn = 0; fn < NB; fn += 16) {
        const v4d t = frag16([&](int m, int k) { return X[m][k]; },
                             [&](int k, int n) { return Q[k][n]; }, 16 * wave, fn, NB);
#pragma unroll
        for (int v = 0; v < 4; ++v) V[(16 * wave + lm) + (long long)(fn + lk + 4 * v) * NB] = t[v];
      }
    }
  }
  if (!rows) return;
  // R2 = W2 X22^T: wave q takes strip q
  {
    const int m = 16 * wave + lm;
    v4d r2[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
    strip_abt<2, HB>(W, 16 * wave, HB, (const double (*)[LP])(X + HB), HB, lane, r2);
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int n = HB + 16 * j + lk + 4 * v;
        if (m < h && n < w) R[(long long)(r0 + m) + (long long)(c0 + n) * ldR] = r2[j][v];
      }
  }
}

}  // namespace panel_dev
}  // namespace adelia
