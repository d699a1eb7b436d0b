// Device kernels of the INLA objective and gradient around the BTA sweeps.
//
// Model (Sec. II-A; Sec. III-B, Eq. 9): every sub-block (i1, i2) of a temporal block is a
// combination of the three spatial base matrices c0, g1, g2:
//   [D_t]^(i1,i2) = sum_s sum_r M_r(t,t)   phi[r][i1][i2][s] * base_s,
//   [B_t]^(i1,i2) = sum_s sum_r M_r(t+1,t) phi[r][i1][i2][s] * base_s,
// with phi[r][i1][i2][s] = sum_m W^(m)_{i1 i2} kappa_m[r][s], W^(m)_{ij} = Li[m][i] Li[m][j]
// (Li = Lambda^-1, Eq. 9) and kappa_m = (K2 coefficients, e^{t_m} K1 coefficients, c0) for
// K1 = e^{2 r_m} c0 + g1, K2 = e^{4 r_m} c0 + 2 e^{2 r_m} g1 + g2.  The univariate model is the
// k = 1 case with W = e^{theta_1}.  Jacobians (Eqs. 10-11): per-field parameters act on kappa_m,
// coupling parameters on W^(m).
//
// Gradient (Sec. III-A-3, Eq. 5), with G^c, G^p the traces of Z = Q^-1 against the base
// matrices (Eq. 6) and q the quadratic forms of x* (Eq. 8):
//   g_k = sum dphi_k . [ M_diag (1/2 (G^p_D - G^c_D - q_D)) + M_off (G^p_B - G^c_B - q_B) ]
//         - 1/2 tau_m sum_o a_o^T Z^c a_o + n_m/2 - tau_m/2 |y_m - A_m x*|^2   (k = tau_m)
//         - theta_k / sigma^2.
#include "common.h"
#include "inla_dev.h"
#include <cmath>

namespace adelia {

namespace {

__device__ __forceinline__ double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  __syncthreads();
  red[tid] = v;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  return red[0];
}

// temporal entry M_r(t, t) (off = 0) or M_r(t+1, t) (off = 1)
__device__ __forceinline__ double tmat(const ModelDev& M, int r, int t, int off) {
  const double* base = M.tm + (long long)r * (2 * M.nt - 1);
  return off ? base[M.nt + t] : base[t];
}

}  // namespace

// ---- per-theta coefficients ------------------------------------------------------------------
__global__ __launch_bounds__(256) void param_kernel(const Models Ms, const double* theta,
                                                    double* phi, double* dphi, double* tau) {
  __shared__ double Li[kMaxFields][kMaxFields];
  __shared__ double dLi[kMaxTheta][kMaxFields][kMaxFields];  // indexed by coupling slot
  __shared__ double k2s[kMaxFields], e3s[kMaxFields];
  const int p = blockIdx.x;
  const ModelDev M = model_at(Ms, p);
  const int k = M.k, d = M.d;
  const double* th = theta + (long long)p * d;
  const int ncoup = k + k * (k - 1) / 2;
  if (threadIdx.x == 0) {
    double Lam[kMaxFields][kMaxFields];
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) Lam[i][j] = 0.0;
    for (int m = 0; m < k; ++m) Lam[m][m] = exp(-0.5 * th[M.idx_prec[m]]);
    int l = 0;
    for (int i = 1; i < k; ++i)
      for (int j = 0; j < i; ++j) Lam[i][j] = th[M.idx_lambda[l++]];
    // Li = Lambda^-1 (lower triangular, forward substitution per column)
    for (int c = 0; c < k; ++c)
      for (int r = 0; r < k; ++r) {
        double s = (r == c) ? 1.0 : 0.0;
        for (int m = c; m < r; ++m) s -= Lam[r][m] * Li[m][c];
        Li[r][c] = (r >= c) ? s / Lam[r][r] : 0.0;
      }
    // dLi = -Li dLambda Li for each coupling slot (prec m, then lambda l)
    for (int cs = 0; cs < ncoup; ++cs) {
      double dL[kMaxFields][kMaxFields];
      for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) dL[i][j] = 0.0;
      if (cs < k) {
        dL[cs][cs] = -0.5 * exp(-0.5 * th[M.idx_prec[cs]]);
      } else {
        int ll = cs - k, ii = 1, jj = 0;
        while (ll > 0) { ++jj; if (jj == ii) { ++ii; jj = 0; } --ll; }
        dL[ii][jj] = 1.0;
      }
      for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
          double s = 0.0;
          for (int a1 = 0; a1 < k; ++a1)
            for (int a2 = 0; a2 < k; ++a2) s += Li[i][a1] * dL[a1][a2] * Li[a2][j];
          dLi[cs][i][j] = -s;
        }
    }
    for (int m = 0; m < k; ++m) {
      k2s[m] = exp(2.0 * th[M.idx_range[m]]);
      e3s[m] = exp(th[M.idx_temporal[m]]);
      tau[(long long)p * k + m] = exp(th[M.idx_tau[m]]);
    }
  }
  __syncthreads();
  const int NE = 9 * k * k;
  for (int e = threadIdx.x; e < NE; e += blockDim.x) {
    const int s = e % 3;
    const int i2 = (e / 3) % k;
    const int i1 = (e / (3 * k)) % k;
    const int r = e / (3 * k * k);
    double kap[kMaxFields], dkr[kMaxFields], dkt[kMaxFields];
    for (int m = 0; m < k; ++m) {
      const double k2 = k2s[m], e3 = e3s[m];
      const double K2[3] = {k2 * k2, 2.0 * k2, 1.0};
      const double K1[3] = {k2, 1.0, 0.0};
      const double dK2[3] = {4.0 * k2 * k2, 4.0 * k2, 0.0};
      const double dK1[3] = {2.0 * k2, 0.0, 0.0};
      if (r == 0) { kap[m] = K2[s]; dkr[m] = dK2[s]; dkt[m] = 0.0; }
      else if (r == 1) { kap[m] = e3 * K1[s]; dkr[m] = e3 * dK1[s]; dkt[m] = e3 * K1[s]; }
      else { kap[m] = (s == 0) ? 1.0 : 0.0; dkr[m] = 0.0; dkt[m] = 0.0; }
    }
    double v = 0.0;
    for (int m = 0; m < k; ++m) v += Li[m][i1] * Li[m][i2] * kap[m];
    phi[(long long)p * NE + e] = v;
    for (int q = 0; q < d; ++q) {
      const int kind = M.role_kind[q], idx = M.role_idx[q];
      double dv = 0.0;
      if (kind == ROLE_RANGE) {
        dv = Li[idx][i1] * Li[idx][i2] * dkr[idx];
      } else if (kind == ROLE_TEMPORAL) {
        dv = Li[idx][i1] * Li[idx][i2] * dkt[idx];
      } else if (kind == ROLE_COUPLING) {
        for (int m = 0; m < k; ++m)
          dv += (dLi[idx][m][i1] * Li[m][i2] + Li[m][i1] * dLi[idx][m][i2]) * kap[m];
      }
      dphi[((long long)p * d + q) * NE + e] = dv;
    }
  }
}

// ---- assembly ----------------------------------------------------------------------------------
// Fills block td of D (if td >= 0) and block tb of B (if tb >= 0) for every chain, one
// 64-lane workgroup per column q: the lanes zero the column (coalesced), then write the
// base-matrix entries of the column in parallel (distinct rows), and lane 0 adds the
// observation term tau_m a_o a_o^T for Qc chains (z even) in a fixed order.
__global__ __launch_bounds__(64) void assemble_blocks_kernel(const Models Ms, int td, int tb,
                                                             double* D, long long zD,
                                                             double* B, long long zB,
                                                             long long ldB, const double* phi,
                                                             const double* tau) {
  const int z = blockIdx.z;
  const int p = z >> 1;
  const ModelDev M = model_at(Ms, p);
  const bool qc = (z & 1) == 0;
  const int b = M.b, ns = M.ns, k = M.k;
  const int q = blockIdx.x;
  const int lane = threadIdx.x;
  // an instance of an uneven batch with fewer blocks: nothing past its last block, and the
  // coupling block after it is zero (the sweep then treats that block as a last block)
  if (td >= M.nt) td = -1;
  double* Dc = td >= 0 ? D + (long long)z * zD + (long long)q * b : nullptr;
  double* Bc = tb >= 0 ? B + (long long)z * zB + (long long)q * ldB : nullptr;
  for (int r = lane; r < b; r += 64) {
    if (Dc) Dc[r] = 0.0;
    if (Bc) Bc[r] = 0.0;
  }
  if (tb >= M.nt - 1) Bc = nullptr;
  __syncthreads();
  const int i2 = q / ns, qq = q % ns;
  const int NE = 9 * k * k;
  const double* ph = phi + (long long)p * NE;
  const int e0 = M.uptr[qq], e1 = M.uptr[qq + 1];
  for (int i1 = 0; i1 < k; ++i1) {
    double cD[3] = {0.0, 0.0, 0.0}, cB[3] = {0.0, 0.0, 0.0};
    for (int r = 0; r < 3; ++r)
      for (int s = 0; s < 3; ++s) {
        const double f = ph[((r * k + i1) * k + i2) * 3 + s];
        if (Dc) cD[s] += tmat(M, r, td, 0) * f;
        if (Bc) cB[s] += tmat(M, r, tb, 1) * f;
      }
    for (int e = e0 + lane; e < e1; e += 64) {
      const long long row = (long long)i1 * ns + M.uidx[e];
      const double v0 = M.uval[e], v1 = M.uval[M.nnz + e], v2 = M.uval[2 * M.nnz + e];
      if (Dc) Dc[row] = cD[0] * v0 + cD[1] * v1 + cD[2] * v2;
      if (Bc) Bc[row] = cB[0] * v0 + cB[1] * v1 + cB[2] * v2;
    }
  }
  __syncthreads();
  if (Dc && qc && lane == 0) {
    const long long g = (long long)td * b + q;
    for (int j = M.colptr[g]; j < M.colptr[g + 1]; ++j) {
      const int o = M.col_o[j];
      const double wq = M.obs_w[4 * o + M.col_e[j]];
      const int m = M.obs_f[o];
      const double tq = tau[(long long)p * k + m] * wq;
      for (int e = 0; e < 4; ++e) {
        const long long row = (long long)m * ns + M.obs_node[4 * o + e];
        Dc[row] += tq * M.obs_w[4 * o + e];
      }
    }
  }
}

// Arrow rows of every block: C_t = sum_o tau X_o^T a_o (rows 0..a-1) and the rhs row
// r_t = sum_o tau y_o a_o (row a); zero for the prior chains.
__global__ __launch_bounds__(256) void assemble_arrow_kernel(const Models Ms, double* C,
                                                             long long zC, long long nb, int ap,
                                                             const double* tau) {
  const int z = blockIdx.z;
  const int p = z >> 1;
  const ModelDev M = model_at(Ms, p);
  const bool qc = (z & 1) == 0;
  const long long g = blockIdx.x * 256LL + threadIdx.x;
  // nb: the columns of the layout (n * b of the largest instance of an uneven batch); the
  // columns past this instance's blocks are zero
  if (g >= nb) return;
  const long long total = (long long)M.nt * M.b;
  const int a = M.a;
  // element (c, q) of block t at t*ap*b + q*ap + c == g*ap + c; one arrow row at a time over
  // the few observations of the column (no per-thread array indexed at run time)
  double* Cz = C + (long long)z * zC + g * ap;
  const int j0 = (qc && g < total) ? M.colptr[g] : 0, j1 = (qc && g < total) ? M.colptr[g + 1] : 0;
  for (int c = 0; c < ap; ++c) {
    double acc = 0.0;
    for (int j = j0; j < j1; ++j) {
      const int o = M.col_o[j];
      const double tw = tau[(long long)p * M.k + M.obs_f[o]] * M.obs_w[4 * o + M.col_e[j]];
      acc += tw * (c < a ? M.X[(long long)o * a + c] : M.y[o]);
    }
    Cz[c] = acc;
  }
}

// Arrowhead tip entries (r >= c) of the ap x ap tip, one workgroup per entry.
__global__ __launch_bounds__(256) void assemble_tip_kernel(const Models Ms, double* T,
                                                           long long zT, int ap,
                                                           const double* tau) {
  __shared__ double red[256];
  const int z = blockIdx.z;
  const int p = z >> 1;
  const ModelDev M = model_at(Ms, p);
  const bool qc = (z & 1) == 0;
  const int r = blockIdx.x % ap, c = blockIdx.x / ap;
  if (r < c) return;
  const int a = M.a;
  double s = 0.0;
  if (qc && c < a) {
    for (int o = threadIdx.x; o < M.n_obs; o += 256) {
      const double t = tau[(long long)p * M.k + M.obs_f[o]];
      const double xr = (r < a) ? M.X[(long long)o * a + r] : M.y[o];
      s += t * xr * M.X[(long long)o * a + c];
    }
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    double v = s;
    if (r == c && r < a) v += M.tip;
    T[(long long)z * zT + r + (long long)c * ap] = (c < a) ? v : 0.0;  // corner starts at 0
  }
}

// ---- Phase A / C traces of one selected-inverse block ------------------------------------------
// grid.x: for each of Z_D and Z_B, k*k sub-block pairs x nch_rows slices of kTraceRows pattern
// rows (<Z^(i1,i2), base_s> restricted to the slice), then k fields x nch_obs slices of
// kTraceObs observations (sum_o a_o^T Zhat a_o).  Every workgroup writes one partial sum per
// quantity; grad_kernel adds the slices in order.
__global__ __launch_bounds__(256) void trace_kernel(const Models Ms, int j, const double* ZD,
                                                    long long zZD, const double* ZB,
                                                    long long zZB, const double* ZC,
                                                    long long zZC, const double* ZT,
                                                    long long zZT, double* TD, double* TB,
                                                    double* O, long long zTr, long long zO) {
  __shared__ double red[256];
  const int z = blockIdx.z;
  const ModelDev M = model_at(Ms, z >> 1);
  const int k = M.k, ns = M.ns, b = M.b, a = M.a;
  const int w = blockIdx.x;
  const int kk = k * k, nr = M.nch_rows;
  // past the instance's blocks or observation slices (uneven batch): nothing to add
  if (j >= M.nt || w >= 2 * kk * nr + k * M.nch_obs) return;
  if (w < 2 * kk * nr) {
    const bool isB = w >= kk * nr;
    const int pair = (w % (kk * nr)) / nr, ch = w % nr;
    const int i1 = pair / k, i2 = pair % k;
    const double* Z = isB ? ZB : ZD;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    const int pr = ch * kTraceRows + (threadIdx.x >> 2);
    if ((!isB || j < M.nt - 1) && pr < ns) {
      Z += (long long)z * (isB ? zZB : zZD);
      const long long row = (long long)i1 * ns + pr;
      for (int e = M.uptr[pr] + (threadIdx.x & 3); e < M.uptr[pr + 1]; e += 4) {
        const double v = Z[row + ((long long)i2 * ns + M.uidx[e]) * b];
        s0 += v * M.uval[e];
        s1 += v * M.uval[M.nnz + e];
        s2 += v * M.uval[2 * M.nnz + e];
      }
    }
    s0 = block_sum(s0, red);
    s1 = block_sum(s1, red);
    s2 = block_sum(s2, red);
    if (threadIdx.x == 0) {
      double* out = (isB ? TB : TD) + (long long)z * zTr + ((long long)j * kk + pair) * 3 * nr + ch;
      out[0] = s0;
      out[nr] = s1;
      out[2 * nr] = s2;
    }
    return;
  }
  // the observation traces enter the gradient through the likelihood precision of Qc only
  if (z & 1) return;
  const int no = M.nch_obs;
  const int m = (w - 2 * kk * nr) / no, ch = (w - 2 * kk * nr) % no;
  const double* Zd = ZD + (long long)z * zZD;
  const double* Zc = a ? ZC + (long long)z * zZC : nullptr;
  const double* Zt = a ? ZT + (long long)z * zZT : nullptr;
  double s = 0.0;
  const int o = M.obs_off[j * k + m] + ch * kTraceObs + (threadIdx.x >> 4);
  if (o < M.obs_off[j * k + m + 1]) {
    // the 16 + 4a + a^2 products of a_o^T Zhat a_o, spread over the observation's 16 lanes
    const double* xo = M.X + (long long)o * a;
    const int nterm = 16 + 4 * a + a * a;
    for (int q = threadIdx.x & 15; q < nterm; q += 16) {
      if (q < 16) {
        const int e = q >> 2, e2 = q & 3;
        const long long g = (long long)m * ns + M.obs_node[4 * o + e];
        const long long g2 = (long long)m * ns + M.obs_node[4 * o + e2];
        s += M.obs_w[4 * o + e] * M.obs_w[4 * o + e2] * Zd[g + g2 * b];
      } else if (q < 16 + 4 * a) {
        const int r = q - 16, e = r / a, c = r % a;
        const long long g = (long long)m * ns + M.obs_node[4 * o + e];
        s += 2.0 * M.obs_w[4 * o + e] * xo[c] * Zc[c + g * a];
      } else {
        const int r = q - 16 - 4 * a, c = r / a, c2 = r % a;
        s += xo[c] * xo[c2] * Zt[c + (long long)c2 * a];
      }
    }
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) O[(long long)z * zO + ((long long)j * k + m) * no + ch] = s;
}

// ---- Phase B: quadratic forms of the mode (Eq. 8) and the data residual -----------------------
__global__ __launch_bounds__(256) void phaseb_kernel(const Models Ms, const double* x,
                                                     long long zxp, double* qD, double* qB,
                                                     long long zq) {
  __shared__ double red[256];
  const ModelDev M = model_at(Ms, blockIdx.z);
  if ((int)blockIdx.x >= M.nt * M.k) return;  // past the instance's blocks (uneven batch)
  // grid.z: theta point (x of its Qc chain at x + z * zxp; outputs at z * zq)
  x += blockIdx.z * zxp;
  qD += blockIdx.z * zq;
  qB += blockIdx.z * zq;
  const int k = M.k, ns = M.ns, b = M.b;
  const int t = blockIdx.x / k, i2 = blockIdx.x % k;
  const bool hasB = t < M.nt - 1;
  double aD[kMaxFields][3], aB[kMaxFields][3];
  for (int i = 0; i < k; ++i)
    for (int s = 0; s < 3; ++s) aD[i][s] = aB[i][s] = 0.0;
  const double* xt = x + (long long)t * b;
  for (int pr = threadIdx.x; pr < ns; pr += 256) {
    double u0 = 0.0, u1 = 0.0, u2 = 0.0;
    for (int e = M.uptr[pr]; e < M.uptr[pr + 1]; ++e) {
      const double xv = xt[(long long)i2 * ns + M.uidx[e]];
      u0 += M.uval[e] * xv;
      u1 += M.uval[M.nnz + e] * xv;
      u2 += M.uval[2 * M.nnz + e] * xv;
    }
    for (int i1 = 0; i1 < k; ++i1) {
      const double xa = xt[(long long)i1 * ns + pr];
      aD[i1][0] += xa * u0; aD[i1][1] += xa * u1; aD[i1][2] += xa * u2;
      if (hasB) {
        const double xb = xt[b + (long long)i1 * ns + pr];
        aB[i1][0] += xb * u0; aB[i1][1] += xb * u1; aB[i1][2] += xb * u2;
      }
    }
  }
  for (int i1 = 0; i1 < k; ++i1)
    for (int s = 0; s < 3; ++s) {
      const double vD = block_sum(aD[i1][s], red);
      const double vB = block_sum(aB[i1][s], red);
      if (threadIdx.x == 0) {
        const long long off = ((long long)t * k * k + i1 * k + i2) * 3 + s;
        qD[off] = vD;
        qB[off] = vB;
      }
    }
}

__global__ __launch_bounds__(256) void resid_kernel(const Models Ms, const double* x,
                                                    long long zxp, int nlay, double* resid,
                                                    long long zr) {
  __shared__ double red[256];
  const ModelDev M = model_at(Ms, blockIdx.z);
  if ((int)blockIdx.x >= M.k * M.nch_resid) return;  // past the instance's slices
  // grid.z: theta point (x of its Qc chain at x + z * zxp; partial sums at z * zr)
  x += blockIdx.z * zxp;
  resid += blockIdx.z * zr;
  // grid.x = k fields x nch_resid slices of kResidObs observations; one partial sum each
  const int m = blockIdx.x / M.nch_resid, ch = blockIdx.x % M.nch_resid;
  const int a = M.a, b = M.b, ns = M.ns;
  const double* xT = x + (long long)nlay * b;  // x: nlay blocks (the layout's), then the tip
  double s = 0.0;
  const int oend = min(M.n_obs, (ch + 1) * kResidObs);
  for (int o = ch * kResidObs + threadIdx.x; o < oend; o += 256) {
    if (M.obs_f[o] != m) continue;
    const long long base = (long long)M.obs_t[o] * b + (long long)m * ns;
    double yh = 0.0;
    for (int e = 0; e < 4; ++e) yh += M.obs_w[4 * o + e] * x[base + M.obs_node[4 * o + e]];
    for (int c = 0; c < a; ++c) yh += M.X[(long long)o * a + c] * xT[c];
    const double rr = M.y[o] - yh;
    s += rr * rr;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) resid[blockIdx.x] = s;
}

__device__ double objective_value(const ModelDev& M, const double* th, const double* tau,
                                  double ldc, double ldp, double zsq) {
  double yy = 0.0, lt = 0.0;
  for (int m = 0; m < M.k; ++m) {
    yy += tau[m] * M.yy[m];
    lt += 0.5 * M.nobs_field[m] * th[M.idx_tau[m]];
  }
  const double s2 = M.sigma * M.sigma;
  double lp = -0.5 * M.d * log(2.0 * M_PI * s2);
  for (int q = 0; q < M.d; ++q) lp -= th[q] * th[q] / (2.0 * s2);
  return 0.5 * ldp - 0.5 * ldc - 0.5 * (yy - zsq) + lt - 0.5 * M.n_obs * log(2.0 * M_PI) + lp;
}

// f for every theta point; chain 2p is Qc, 2p+1 is Qp.
__global__ void objective_kernel(const Models Ms, const double* theta, int batch,
                                 const double* tau, const double* ld, const double* zsq,
                                 const int32_t* info, double* f, int32_t* info_out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= batch) return;
  const ModelDev M = model_at(Ms, p);
  f[p] = objective_value(M, theta + (long long)p * M.d, tau + (long long)p * M.k, ld[2 * p],
                         ld[2 * p + 1], zsq[2 * p]);
  const int32_t ic = info[2 * p], ip = info[2 * p + 1];
  info_out[p] = (ic != 0 && ic != INT32_MAX) ? ic : ((ip != INT32_MAX) ? ip : 0);
}

// Gradient assembly, one workgroup per theta point p (chains 2p = Qc, 2p + 1 = Qp).  Optionally
// (one point) writes the decomposition terms = [f, log|Qp|, log|Qc|, |z|^2, tr(Z_T of Qc),
// PhaseA(d), PhaseB(d), PhaseC(d), dlog l(d), dlog p(d), grad(d)].
__global__ __launch_bounds__(256) void grad_kernel(const Models Ms, const double* theta,
                                                   const double* dphi, const double* tau,
                                                   const double* TD, const double* TB,
                                                   long long zTr, const double* O, long long zO,
                                                   const double* qD, const double* qB,
                                                   long long zq, const double* resid,
                                                   long long zr, const double* ld,
                                                   const double* zsq, const double* ZTc,
                                                   long long zZT, const int32_t* info,
                                                   double* f, double* grad, int32_t* info_out,
                                                   double* terms) {
  __shared__ double SA[9 * kMaxFields * kMaxFields];
  __shared__ double SB[9 * kMaxFields * kMaxFields];
  __shared__ double SC[9 * kMaxFields * kMaxFields];
  const int p = blockIdx.x;
  const ModelDev M = model_at(Ms, p);
  const int k = M.k, kk = k * k, nt = M.nt, d = M.d;
  const int NE = 9 * kk;
  theta += (long long)p * d;
  dphi += (long long)p * NE * d;
  tau += (long long)p * k;
  TD += 2LL * p * zTr;
  TB += 2LL * p * zTr;
  O += 2LL * p * zO;
  qD += p * zq;
  qB += p * zq;
  resid += p * zr;
  ld += 2 * p;
  zsq += 2 * p;
  ZTc += 2LL * p * zZT;
  info += 2 * p;
  f += p;
  grad += (long long)p * d;
  info_out += p;
  // Per element e = (r, i1, i2, s): sums over the time steps and the trace slices, spread over
  // the workgroup (each thread takes time steps t = tid, tid + 256, ...; block sums in a fixed
  // order)
  __shared__ double red[256];
  const int nr = M.nch_rows;
  for (int e = 0; e < NE; ++e) {
    const int r = e / (3 * kk);
    const int rest = e % (3 * kk);  // (i1*k + i2)*3 + s
    double a = 0.0, bq = 0.0, c = 0.0;
    for (int t = threadIdx.x; t < nt; t += blockDim.x) {
      const long long o = (long long)t * kk * 3 + rest;
      double td0 = 0.0, td1 = 0.0, tb0 = 0.0, tb1 = 0.0;
      for (int q = 0; q < nr; ++q) {
        td0 += TD[o * nr + q];
        td1 += TD[zTr + o * nr + q];
      }
      const double md = tmat(M, r, t, 0);
      a -= 0.5 * md * td0;
      bq -= 0.5 * md * qD[o];
      c += 0.5 * md * td1;
      if (t < nt - 1) {
        for (int q = 0; q < nr; ++q) {
          tb0 += TB[o * nr + q];
          tb1 += TB[zTr + o * nr + q];
        }
        const double mo = tmat(M, r, t, 1);
        a -= mo * tb0;
        bq -= mo * qB[o];
        c += mo * tb1;
      }
    }
    a = block_sum(a, red);
    bq = block_sum(bq, red);
    c = block_sum(c, red);
    if (threadIdx.x == 0) {
      SA[e] = a;
      SB[e] = bq;
      SC[e] = c;
    }
  }
  __syncthreads();
  const double fval = objective_value(M, theta, tau, ld[0], ld[1], zsq[0]);
  for (int q = threadIdx.x; q < d; q += blockDim.x) {
    double pa = 0.0, pb = 0.0, pc = 0.0, dl = 0.0;
    for (int e = 0; e < NE; ++e) {
      const double w = dphi[(long long)q * NE + e];
      pa += w * SA[e];
      pb += w * SB[e];
      pc += w * SC[e];
    }
    if (M.role_kind[q] == ROLE_TAU) {
      const int m = M.role_idx[q];
      double so = 0.0;
      for (int t = 0; t < nt; ++t)
        for (int c = 0; c < M.nch_obs; ++c) so += O[((long long)t * k + m) * M.nch_obs + c];
      pa += -0.5 * tau[m] * so;
      double rs = 0.0;
      for (int c = 0; c < M.nch_resid; ++c) rs += resid[m * M.nch_resid + c];
      dl = 0.5 * M.nobs_field[m] - 0.5 * tau[m] * rs;
    }
    const double dp = -theta[q] / (M.sigma * M.sigma);
    const double g = pa + pb + pc + dl + dp;
    grad[q] = g;
    if (terms) {
      terms[5 + q] = pa;
      terms[5 + d + q] = pb;
      terms[5 + 2 * d + q] = pc;
      terms[5 + 3 * d + q] = dl;
      terms[5 + 4 * d + q] = dp;
      terms[5 + 5 * d + q] = g;
    }
  }
  if (threadIdx.x == 0) {
    f[0] = fval;
    const int32_t ic = info[0], ip = info[1];
    info_out[0] = (ic != 0 && ic != INT32_MAX) ? ic : ((ip != INT32_MAX) ? ip : 0);
    if (terms) {
      double tr = 0.0;
      for (int c = 0; c < M.a; ++c) tr += ZTc[c + (long long)c * M.a];
      terms[0] = fval;
      terms[1] = ld[1];
      terms[2] = ld[0];
      terms[3] = zsq[0];
      terms[4] = tr;
    }
  }
}

// ---- the two-sided split ---------------------------------------------------------------------
// Chains of the halves: 0, 1 = half A's Qc, Qp; 2, 3 = half B's.  zn[z]: blocks swept by chain
// z (its separator block is local block zn[z]).

// The reduced system's block, arrow rows and tip (chain 0 = Qc, 1 = Qp): the sums of the two
// halves' Schur-complemented separator blocks, separator arrow rows and tips.
__global__ void split_merge_kernel(const double* D, long long zD, long long sD, int slotsD,
                                   const double* C, long long zC, long long sC, const double* T,
                                   long long zT, const int32_t* zn, int b, int ap, double* Dr,
                                   long long zDr, double* Cr, long long zCr, double* Tr,
                                   long long zTr) {
  const int mat = blockIdx.z;
  const int zA = mat, zB = 2 + mat;
  const long long bb = (long long)b * b, cb = (long long)ap * b, tt = (long long)ap * ap;
  const double* DA = D + zA * zD + (long long)(zn[zA] % slotsD) * sD;
  const double* DB = D + zB * zD + (long long)(zn[zB] % slotsD) * sD;
  const double* CA = C + zA * zC + (long long)zn[zA] * sC;
  const double* CB = C + zB * zC + (long long)zn[zB] * sC;
  const double* TA = T + zA * zT;
  const double* TB = T + zB * zT;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < bb + cb + tt;
       e += (long long)gridDim.x * 256) {
    if (e < bb)
      Dr[mat * zDr + e] = DA[e] + DB[e];
    else if (e < bb + cb)
      Cr[mat * zCr + (e - bb)] = CA[e - bb] + CB[e - bb];
    else
      Tr[mat * zTr + (e - bb - cb)] = TA[e - bb - cb] + TB[e - bb - cb];
  }
}

// The reduced system's selected inverse and mode seed both halves: Z_D and Z_C of the
// separator go into each half chain's slots of its local block zn[z], Z_T into its tip, x of
// the separator into its block zn[z] of x and x_T into its tip part.
__global__ void split_seed_kernel(const double* ZDr, long long zZDr, const double* ZCr,
                                  long long zZCr, const double* ZTr, long long zZTr,
                                  const double* xr, long long zxr, const double* xTr,
                                  long long zxTr, int b, int a, const int32_t* zn, int slotsZD,
                                  double* ZD, long long zZD, double* ZC, long long zZC,
                                  double* ZT, long long zZT, double* x, long long zx, double* xT,
                                  long long zxT) {
  const int z = blockIdx.z, mat = z & 1;
  const long long bb = (long long)b * b, cb = (long long)a * b;
  const int j = zn[z];
  double* zd = ZD + z * zZD + (long long)(j % slotsZD) * bb;
  double* zc = ZC + z * zZC + (long long)(j % 2) * cb;
  const long long tot = bb + cb + (long long)a * a + b + a;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < tot; e += (long long)gridDim.x * 256) {
    if (e < bb) {
      zd[e] = ZDr[mat * zZDr + e];
    } else if (e < bb + cb) {
      zc[e - bb] = ZCr[mat * zZCr + (e - bb)];
    } else if (e < bb + cb + (long long)a * a) {
      ZT[z * zZT + (e - bb - cb)] = ZTr[mat * zZTr + (e - bb - cb)];
    } else if (e < bb + cb + (long long)a * a + b) {
      const long long i = e - bb - cb - (long long)a * a;
      x[z * zx + (long long)j * b + i] = xr[mat * zxr + i];
    } else {
      const long long i = e - bb - cb - (long long)a * a - b;
      xT[z * zxT + i] = xTr[mat * zxTr + i];
    }
  }
}

__device__ __forceinline__ bool failed(int32_t v) { return v != 0 && v != INT32_MAX; }

// f from the log-determinants of the halves and of the reduced system and |z|^2 of the reduced
// tip, the gradient as the sum of the halves' gradients (gv: 2 x d, or null for f alone), and
// the first failure of any chain (its column numbered within its own chain).
__global__ void split_combine_kernel(const Models Ms, const double* theta, const double* tau,
                                     const double* ldh, const double* ldr, const double* zsqr,
                                     const int32_t* infh, const int32_t* infr, const double* gv,
                                     const int32_t* ginfo, double* f, double* grad,
                                     int32_t* info) {
  const ModelDev M = model_at(Ms, 0);
  const int d = M.d;
  for (int q = threadIdx.x; q < d && gv; q += blockDim.x) grad[q] = gv[q] + gv[d + q];
  if (threadIdx.x == 0) {
    const double ldc = ldh[0] + ldh[2] + ldr[0], ldp = ldh[1] + ldh[3] + ldr[1];
    f[0] = objective_value(M, theta, tau, ldc, ldp, zsqr[0]);
    int32_t v = 0;
    for (int z = 0; z < 4 && !v; ++z) if (failed(infh[z])) v = infh[z];
    for (int z = 0; z < 2 && !v; ++z) if (failed(infr[z])) v = infr[z];
    for (int z = 0; z < 2 && !v && ginfo; ++z) if (failed(ginfo[z])) v = ginfo[z];
    info[0] = v;
  }
}

__global__ void yy_kernel(const ModelDev M, double* yy) {
  __shared__ double red[256];
  const int m = blockIdx.x;
  double s = 0.0;
  for (int o = threadIdx.x; o < M.n_obs; o += 256)
    if (M.obs_f[o] == m) s += M.y[o] * M.y[o];
  s = block_sum(s, red);
  if (threadIdx.x == 0) yy[m] = s;
}

__global__ void stencil_kernel(const double* theta, int d, double h, double* Th) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int npts = 2 * d + 1;
  if (i >= npts * d) return;
  const int p = i / d, q = i % d;
  double v = theta[q];
  if (p > 0) {
    const int j = (p - 1) / 2;
    if (j == q) v += ((p - 1) % 2 == 0) ? h : -h;
  }
  Th[i] = v;
}

__global__ void fd_kernel(const double* fv, int d, double h, double* f, double* grad) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j == 0) f[0] = fv[0];
  if (j < d) grad[j] = (fv[1 + 2 * j] - fv[2 + 2 * j]) / (2.0 * h);
}

// W_t = B_t Y with Y = G_t^T G_t = (L_Dt L_Dt^T)^-1 (so W_t = L_Bt G_t, the b rows of [W; V] in
// the selected inversion), B_t = Q[t+1, t] sparse (the base-matrix pattern for every field
// pair, as assembled).  The workgroups of a chain walk batches of cb columns: the batch's
// columns of Y (stored in full) are loaded into LDS, then each row of B_t, its pattern and
// values read once per batch, is applied to all of them.  Bound by the pattern reads (b/cb
// passes over B_t) and by reading Y and writing W once: 16 b^2 bytes per chain.
__global__ __launch_bounds__(256) void w_from_gtg_kernel(const Models Ms, int t, int zdiv,
                                                         const int32_t* zn, const double* Y,
                                                         long long zY, double* W, long long zW,
                                                         const double* phi, int cb) {
  extern __shared__ double ys[];  // cb columns of Y, b each
  __shared__ double cB[kMaxFields][kMaxFields][3];
  const int z = blockIdx.z;
  if (zdiv > 0) t = z % zdiv;
  if (z_idle(zn, t, zdiv, z)) return;
  const int p = (zdiv > 0 ? z / zdiv : z) >> 1;
  const ModelDev M = model_at(Ms, p);
  const int b = M.b, ns = M.ns, k = M.k;
  const double* Yz = Y + (long long)z * zY;
  if (t >= M.nt - 1) {
    // no coupling block after the instance's last block (uneven batch): W_t = 0
    double* Wz = W + (long long)z * zW;
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < (long long)b * b;
         e += (long long)gridDim.x * 256)
      Wz[e] = 0.0;
    return;
  }
  if (threadIdx.x < k * k * 3) {
    const int s = threadIdx.x % 3, i2 = (threadIdx.x / 3) % k, i1 = threadIdx.x / (3 * k);
    const double* ph = phi + (long long)p * 9 * k * k;
    double v = 0.0;
    for (int r = 0; r < 3; ++r) v += tmat(M, r, t, 1) * ph[((r * k + i1) * k + i2) * 3 + s];
    cB[i1][i2][s] = v;
  }
  // the workgroups of a chain walk batches of cb columns; each row of B_t (its pattern read
  // once per batch) is applied to all of them
  for (int c0 = blockIdx.x * cb; c0 < b; c0 += gridDim.x * cb) {
    const int nc = min(cb, b - c0);
    __syncthreads();  // the previous batch's reads of ys are done (and cB is written)
    for (int e = threadIdx.x; e < nc * b; e += 256) ys[e] = Yz[(long long)c0 * b + e];
    __syncthreads();
    double* Wc = W + (long long)z * zW + (long long)c0 * b;
    for (int row = threadIdx.x; row < b; row += 256) {
      const int i1 = row / ns, rr = row % ns;
      double acc[kWBatch];
#pragma unroll
      for (int cc = 0; cc < kWBatch; ++cc) acc[cc] = 0.0;
      for (int e = M.uptr[rr]; e < M.uptr[rr + 1]; ++e) {
        const int qq = M.uidx[e];
        const double v0 = M.uval[e], v1 = M.uval[M.nnz + e], v2 = M.uval[2 * M.nnz + e];
        for (int i2 = 0; i2 < k; ++i2) {
          const double bv = cB[i1][i2][0] * v0 + cB[i1][i2][1] * v1 + cB[i1][i2][2] * v2;
          const double* yq = ys + i2 * ns + qq;
#pragma unroll
          for (int cc = 0; cc < kWBatch; ++cc)
            if (cc < nc) acc[cc] += bv * yq[(long long)cc * b];
        }
      }
#pragma unroll
      for (int cc = 0; cc < kWBatch; ++cc)
        if (cc < nc) Wc[(long long)cc * b + row] = acc[cc];
    }
  }
}

// W_t = B_t Y, the product of w_from_gtg_kernel, with the pattern held in registers.  A
// workgroup owns a tile of kWRows pattern rows rr (for every field i1: the rows i1 ns + rr of
// W_t) and a slice of the columns; each thread keeps its pattern row's entries (column offsets
// and the values of the three base matrices, padded with zeros to kWDeg) for the whole kernel.
// The tile's rows touch pattern columns [lo, hi) only (a band, per field of Y), so cb columns of
// those rows of Y go through LDS at a time, column-major with the band rows contiguous: the
// threads of a wave read neighbouring addresses.  For each column a thread forms the three
// base-matrix products T_s(i2) = sum_e U_s(rr, e) Y(i2 ns + qq_e, c) for every field i2 of Y and
// combines them with the coupling coefficients: W_t(i1 ns + rr, c) =
// sum_{i2, s} cB(i1, i2, s) T_s(i2).  Bound by reading Y's bands and writing W_t once.
template <int KF>
__global__ __launch_bounds__(256) void w_band_kernel(const Models Ms, int t, int zdiv,
                                                     const int32_t* zn, const double* Y,
                                                     long long zY, double* W, long long zW,
                                                     const double* phi, int cb, int cs) {
  extern __shared__ double ys[];  // k x cb x bw: (field, column, band row), band row fastest
  __shared__ double cB[KF][KF][3];
  const int z = blockIdx.z;
  if (zdiv > 0) t = z % zdiv;
  if (z_idle(zn, t, zdiv, z)) return;
  const int p = (zdiv > 0 ? z / zdiv : z) >> 1;
  const ModelDev M = model_at(Ms, p);
  const int b = M.b, ns = M.ns, k = M.k;
  const int r0 = blockIdx.x * kWRows;
  if (r0 >= ns) return;  // a tile past this instance's pattern (uniform over the workgroup)
  const int rr = r0 + threadIdx.x;
  const bool act = rr < ns;
  const int c0s = blockIdx.y * cs, c1s = min(b, c0s + cs);
  const double* Yz = Y + (long long)z * zY;
  double* Wz = W + (long long)z * zW;
  if (t >= M.nt - 1) {
    // no coupling block after the instance's last block (uneven batch): W_t = 0
    if (act)
      for (int c = c0s; c < c1s; ++c)
        for (int i1 = 0; i1 < k; ++i1) Wz[(long long)c * b + i1 * ns + rr] = 0.0;
    return;
  }
  if (threadIdx.x < k * k * 3) {
    const int sidx = threadIdx.x % 3, i2 = (threadIdx.x / 3) % k, i1 = threadIdx.x / (3 * k);
    const double* ph = phi + (long long)p * 9 * k * k;
    double v = 0.0;
    for (int r = 0; r < 3; ++r) v += tmat(M, r, t, 1) * ph[((r * k + i1) * k + i2) * 3 + sidx];
    cB[i1][i2][sidx] = v;
  }
  const int lo = M.wband[2 * blockIdx.x], bw = M.wband[2 * blockIdx.x + 1] - lo;
  int off[kWDeg];
  double u0[kWDeg], u1[kWDeg], u2[kWDeg];
  {
    const int e0 = act ? M.uptr[rr] : 0;
    const int ne = act ? M.uptr[rr + 1] - e0 : 0;
#pragma unroll
    for (int e = 0; e < kWDeg; ++e) {
      const bool ok = e < ne;
      const int ee = ok ? e0 + e : 0;
      off[e] = ok ? M.uidx[ee] - lo : 0;
      u0[e] = ok ? M.uval[ee] : 0.0;
      u1[e] = ok ? M.uval[M.nnz + ee] : 0.0;
      u2[e] = ok ? M.uval[2 * M.nnz + ee] : 0.0;
    }
  }
  for (int cc0 = c0s; cc0 < c1s; cc0 += cb) {
    const int nc = min(cb, c1s - cc0);
    __syncthreads();  // the previous batch's reads of ys are done (and cB is written)
    const int tot = k * nc * bw;
    if constexpr (KF >= 3) {
      // column by column (k >= 3: the products take the registers two waves per SIMD leave)
      for (int ic = 0; ic < k * nc; ++ic) {
        const int i2 = ic / nc, c = ic % nc;
        const double* src = Yz + (long long)(cc0 + c) * b + i2 * ns + lo;
        double* dst = ys + (i2 * cb + c) * bw;
        for (int q = threadIdx.x; q < bw; q += 256) dst[q] = src[q];
      }
    } else {
      // the pass's k nc bw band entries, eight per thread in flight at a time (neighbouring
      // threads read neighbouring rows of one column of Y); the column-by-column loop waited
      // for each column's loads in turn (b = 1024, 104 blocks: 1099 -> 737 us)
      for (int e0 = 0; e0 < tot; e0 += 8 * 256) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = min(e0 + u * 256 + (int)threadIdx.x, tot - 1);
          const int ic = e / bw, q = e - ic * bw, i2 = ic / nc, c = ic - i2 * nc;
          v[u] = Yz[(long long)(cc0 + c) * b + i2 * ns + lo + q];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = e0 + u * 256 + (int)threadIdx.x;
          if (e < tot) {
            const int ic = e / bw, q = e - ic * bw, i2 = ic / nc, c = ic - i2 * nc;
            ys[(i2 * cb + c) * bw + q] = v[u];
          }
        }
      }
    }
    __syncthreads();
    if (!act) continue;
    for (int c = 0; c < nc; ++c) {
      double T[3][KF];
#pragma unroll
      for (int i2 = 0; i2 < KF; ++i2) {
        T[0][i2] = 0.0;
        T[1][i2] = 0.0;
        T[2][i2] = 0.0;
        if (i2 < k) {
          const double* yc = ys + (i2 * cb + c) * bw;
#pragma unroll
          for (int e = 0; e < kWDeg; ++e) {
            const double y = yc[off[e]];
            T[0][i2] = fma(u0[e], y, T[0][i2]);
            T[1][i2] = fma(u1[e], y, T[1][i2]);
            T[2][i2] = fma(u2[e], y, T[2][i2]);
          }
        }
      }
#pragma unroll
      for (int i1 = 0; i1 < KF; ++i1) {
        if (i1 >= k) break;
        double w = 0.0;
#pragma unroll
        for (int i2 = 0; i2 < KF; ++i2) {
          if (i2 >= k) break;
          w = fma(cB[i1][i2][0], T[0][i2], w);
          w = fma(cB[i1][i2][1], T[1][i2], w);
          w = fma(cB[i1][i2][2], T[2][i2], w);
        }
        Wz[(long long)(cc0 + c) * b + i1 * ns + rr] = w;
      }
    }
  }
}

template __global__ void w_band_kernel<1>(const Models, int, int, const int32_t*, const double*,
                                          long long, double*, long long, const double*, int, int);
template __global__ void w_band_kernel<2>(const Models, int, int, const int32_t*, const double*,
                                          long long, double*, long long, const double*, int, int);
template __global__ void w_band_kernel<3>(const Models, int, int, const int32_t*, const double*,
                                          long long, double*, long long, const double*, int, int);
template __global__ void w_band_kernel<4>(const Models, int, int, const int32_t*, const double*,
                                          long long, double*, long long, const double*, int, int);

// Points of the second-order central-difference Hessian (2d^2 + 1): 0 the centre; 1 + 2j and
// 2 + 2j the steps +h e_j and -h e_j; then, for each pair j < k in order, four points
// (+e_j + e_k, +e_j - e_k, -e_j + e_k, -e_j - e_k) times h.
__global__ void hess_stencil_kernel(const double* theta, int d, double h, double* Th) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int npts = 2 * d * d + 1;
  if (i >= npts * d) return;
  const int p = i / d, c = i % d;
  double v = theta[c];
  if (p >= 1 && p <= 2 * d) {
    if ((p - 1) / 2 == c) v += ((p - 1) % 2 == 0) ? h : -h;
  } else if (p > 2 * d) {
    int q = (p - 1 - 2 * d) / 4;
    const int r = (p - 1 - 2 * d) % 4;
    int j = 0;
    while (q >= d - 1 - j) {
      q -= d - 1 - j;
      ++j;
    }
    const int k = j + 1 + q;
    if (c == j) v += (r < 2) ? h : -h;
    if (c == k) v += (r % 2 == 0) ? h : -h;
  }
  Th[i] = v;
}

// H (d x d, column-major) from the objective values at hess_stencil_kernel's points.
__global__ void fd_hessian_kernel(const double* fv, int d, double h, double* f, double* H) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) f[0] = fv[0];
  if (i >= d * d) return;
  const int r = i % d, c = i / d;
  double v;
  if (r == c) {
    v = (fv[1 + 2 * r] - 2.0 * fv[0] + fv[2 + 2 * r]) / (h * h);
  } else {
    const int a = r < c ? r : c, b = r < c ? c : r;
    const int base = 1 + 2 * d + 4 * (a * (2 * d - a - 1) / 2 + (b - a - 1));
    v = (fv[base] - fv[base + 1] - fv[base + 2] + fv[base + 3]) / (4.0 * h * h);
  }
  H[i] = v;
}

// Eq. 12: column j of H (d x d, column-major) from the gradients at stencil_kernel's points
// theta + h e_j (point 1 + 2j) and theta - h e_j (point 2 + 2j); f and grad at the centre.
__global__ void grad_hessian_kernel(const double* fv, const double* gv, int d, double h,
                                    double* f, double* grad, double* H) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) f[0] = fv[0];
  if (i < d) grad[i] = gv[i];
  if (i >= d * d) return;
  const int r = i % d, j = i / d;
  H[i] = (gv[(long long)(1 + 2 * j) * d + r] - gv[(long long)(2 + 2 * j) * d + r]) / (2.0 * h);
}

}  // namespace adelia
