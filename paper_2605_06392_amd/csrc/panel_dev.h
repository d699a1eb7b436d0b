// Panel step of the blocked Cholesky of a diagonal block (Sec. III-A-1, Alg. 1, chol()).
//
// The 64 x 64 diagonal tile of panel k is factored, together with its inverse, as two 32 x 32
// leaves: each leaf is eliminated two columns per step by ONE wavefront (registers hold 2 x 2
// sub-blocks, the current column pair travels through LDS; a single wave needs no workgroup
// barrier between steps because its LDS operations complete in program order), and the
// off-diagonal solve L21 = A21 X11^T, the update A22 -= L21 L21^T and the inverse merge
// X21 = -X22 L21 X11 run on the matrix cores across the four waves.  Workgroup x > 0 also
// solves its 64-row tile of the panel as A_jk L_kk^-T.
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
// one that sees the count complete stores L_kk, L_kk^-1, the log-diagonal sum and the pivot
// check (all workgroups compute bit-identical tiles) and resets the counter for the next
// launch.  No workgroup ever waits on another.
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
  // if not null (and upd): the writer also stores V = L_kk^-1 Q (64 x 64, column-major, chain
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

// Columns j0 = 2 JQ and j1 = j0 + 1 of a 16 x 16 leaf held as 2 x 2 blocks, one per lane (lane
// (br, bc) holds rows 2 br.., columns 2 bc..).  The column pair has been published to LDS
// updated but unscaled (cp: column j0 then column j1; xp: rows j0 and j1 of L^-1 before their
// scaling), so every lane factors the 2 x 2 pivot block itself, scales the entries it needs and
// applies the rank-2 update to the trailing part of L and to the rows of L^-1 below j1; then
// the lanes holding pair JQ + 1 publish it.  Masks are selects on the operands: lanes above the
// diagonal compute finite values that are never read.
template <int JQ>
__device__ __forceinline__ void leaf_pair(double (&a)[2][2], double (&x)[2][2], double* cp,
                                          double* xp, double* piv, int o, int br, int bc,
                                          int lane) {
  constexpr int j0 = 2 * JQ, j1 = j0 + 1;
  const double* c0 = cp;
  const double* c1 = cp + QB;
  const double a00 = c0[j0], a10 = c0[j1], a11 = c1[j1];
  double c0r[2], c1r[2], c0c[2], c1c[2], x0c[2], x1c[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    c0r[q] = c0[2 * br + q];
    c1r[q] = c1[2 * br + q];
    c0c[q] = c0[2 * bc + q];
    c1c[q] = c1[2 * bc + q];
    x0c[q] = xp[2 * bc + q];
    x1c[q] = xp[QB + 2 * bc + q];
  }
  double p0, r0, p1, r1;
  pivot(a00, p0, r0);
  const double l10 = a10 * r0;
  const double d1 = fma(-l10, l10, a11);
  pivot(d1, p1, r1);
  if (lane == 0) {
    piv[o + j0] = a00;
    piv[o + j1] = d1;
  }
  const bool rowm = br > JQ, colm = bc > JQ;
  double L0r[2], L1r[2], L0c[2], L1c[2], X0[2], X1[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    L0r[q] = c0r[q] * r0;
    L1r[q] = fma(-L0r[q], l10, c1r[q]) * r1;
    L0c[q] = c0c[q] * r0;
    L1c[q] = fma(-L0c[q], l10, c1c[q]) * r1;
    X0[q] = x0c[q] * r0;
    X1[q] = fma(-l10, X0[q], x1c[q]) * r1;
  }
#pragma unroll
  for (int ii = 0; ii < 2; ++ii) {
    const double u0 = rowm ? L0r[ii] : 0.0, u1 = rowm ? L1r[ii] : 0.0;
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) {
      const double v0 = colm ? L0c[jj] : 0.0, v1 = colm ? L1c[jj] : 0.0;
      a[ii][jj] = fma(-u0, v0, fma(-u1, v1, a[ii][jj]));
      x[ii][jj] = fma(-u0, X0[jj], fma(-u1, X1[jj], x[ii][jj]));
    }
  }
  if (bc == JQ) {
#pragma unroll
    for (int ii = 0; ii < 2; ++ii) {
      a[ii][0] = L0r[ii];
      a[ii][1] = L1r[ii];
    }
  }
  if (br == JQ) {
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) {
      x[0][jj] = X0[jj];
      x[1][jj] = X1[jj];
    }
  }
  wave_order();  // every lane has read pair JQ before it is replaced
  if constexpr (JQ + 1 < QB / 2) {
    if (bc == JQ + 1) {
#pragma unroll
      for (int ii = 0; ii < 2; ++ii) {
        cp[2 * br + ii] = a[ii][0];
        cp[QB + 2 * br + ii] = a[ii][1];
      }
    }
    if (br == JQ + 1) {
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        xp[2 * bc + jj] = x[0][jj];
        xp[QB + 2 * bc + jj] = x[1][jj];
      }
    }
    wave_order();
  }
}

// Factor the 16 x 16 leaf at (o, o) of S (lower triangle, already updated) with one wavefront.
// On exit S holds L (lower, zeros above) and X holds L^-1 on that leaf; piv[o + j] = pivot^2.
__device__ void leaf16(double (*S)[LP], double (*X)[LP], double* cp, double* xp, double* piv,
                       int o) {
  const int lane = threadIdx.x & 63;
  const int br = lane >> 3, bc = lane & 7;
  double a[2][2], x[2][2];
#pragma unroll
  for (int ii = 0; ii < 2; ++ii)
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) {
      const int r = 2 * br + ii, c = 2 * bc + jj;
      const double v = S[o + r][o + c];
      a[ii][jj] = (r >= c) ? v : 0.0;
      x[ii][jj] = (r == c) ? 1.0 : 0.0;
    }
  if (bc == 0) {
#pragma unroll
    for (int ii = 0; ii < 2; ++ii) {
      cp[2 * br + ii] = a[ii][0];
      cp[QB + 2 * br + ii] = a[ii][1];
    }
  }
  if (br == 0) {
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) {
      xp[2 * bc + jj] = x[0][jj];
      xp[QB + 2 * bc + jj] = x[1][jj];
    }
  }
  wave_order();
  leaf_pair<0>(a, x, cp, xp, piv, o, br, bc, lane);
  leaf_pair<1>(a, x, cp, xp, piv, o, br, bc, lane);
  leaf_pair<2>(a, x, cp, xp, piv, o, br, bc, lane);
  leaf_pair<3>(a, x, cp, xp, piv, o, br, bc, lane);
  leaf_pair<4>(a, x, cp, xp, piv, o, br, bc, lane);
  leaf_pair<5>(a, x, cp, xp, piv, o, br, bc, lane);
  leaf_pair<6>(a, x, cp, xp, piv, o, br, bc, lane);
  leaf_pair<7>(a, x, cp, xp, piv, o, br, bc, lane);
#pragma unroll
  for (int ii = 0; ii < 2; ++ii)
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) {
      const int r = 2 * br + ii, c = 2 * bc + jj;
      const bool low = r >= c;
      S[o + r][o + c] = low ? a[ii][jj] : 0.0;
      X[o + r][o + c] = low ? x[ii][jj] : 0.0;
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
__device__ void leaf32(double (*S)[LP], double (*X)[LP], double* col, double* xr, double* piv,
                       int o) {
  const int lane = threadIdx.x & 63;
  const int m = lane & 15, n0 = lane >> 4;
  const int h = o + QB;
  leaf16(S, X, col, xr, piv, o);
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
  leaf16(S, X, col, xr, piv, h);
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
  double col[2 * QB], xr[2 * QB], piv[NB];
  int writer;
};

// One workgroup of a panel launch: workgroup bx of nbx (x index within chain blockIdx.z).
__device__ __forceinline__ void panel_body(const PanelArgs& P, int bx, int nbx, PanelSmem& sm) {
  double (*S)[LP] = sm.S;
  double (*X)[LP] = sm.X;
  double (*Q)[LP] = sm.Q;
  double (*W)[LP] = sm.W;
  double* col = sm.col;
  double* xr = sm.xr;
  double* piv = sm.piv;
  int& writer = sm.writer;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lm = lane & 15, lk = lane >> 4;
  const int z = blockIdx.z;
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
    leaf32(S, X, col, xr, piv, 0);
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
    leaf32(S, X, col, xr, piv, HB);
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

  if (writer) {
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
    for (int e = tid; e < w * w; e += 256) {
      const int r = e % w, c = e / w;
      const long long off = (long long)(c0 + r) + (long long)(c0 + c) * b;
      D[off] = (r >= c) ? S[r][c] : 0.0;
      G[off] = (r >= c) ? X[r][c] : 0.0;
    }
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
