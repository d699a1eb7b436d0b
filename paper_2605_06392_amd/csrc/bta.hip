// Host orchestration of the BTA sweeps.  Every launch covers all `nz` chains of a batch
// (grid.z), so a gradient (Qc and Qp) or a finite-difference stencil (2 chains per theta)
// runs its block steps as single launches.
//
// Forward (Sec. III-A-1, Alg. 1), per block i:
//   1. chol(D_i) by 64-wide panels (panel.hip) plus trailing GEMM updates.  The rows [B_i; C~_i]
//      are stacked under the block and solved with the same panels (the TRSM of Alg. 1), so
//      every panel launch and trailing update also covers them and [L_Bi; L_Ci] comes out of
//      the factorisation.  The right-hand side travels as an extra arrow row (C~_i's last row
//      is r~_i^T), so L_Ci's last row is z_i^T -- the forward solve fused into the sweep.  The
//      panel kernels leave the 64 x 64 diagonal inverses in G_i.
//   2. When the inverse is needed (solve, selected inversion), G_i = L_Di^-1 is completed by
//      recursive doubling: X21 = -X22 L21 X11 (two GEMMs per level).
//   3. [[D_{i+1}], [C~_{i+1}, T~]] -= [L_Bi; L_Ci][L_Bi; L_Ci]^T: one lower-triangular GEMM
//      updating the next diagonal block, the next arrow block (and r~_{i+1}), the tip (and
//      v_T, and -|z_i|^2 in the tip's corner).
// Selected inversion (Sec. III-A, Phase A; the recurrence follows from Sigma L = L^-T):
//   [W; V] = [L_Bj; L_Cj] G_j,
//   [Z_Bj; Z_Cj] = -[[Z_D{j+1}, Z_C{j+1}^T], [Z_C{j+1}, Z_T]] [W; V],
//   Z_Dj = G_j^T G_j - [Z_Bj; Z_Cj]^T [W; V].
#include "common.h"
#include "launchers.h"
#include <algorithm>

namespace adelia {

static inline long long blk_off(int t, int slots, long long bb) { return (long long)(t % slots) * bb; }

// CUs of the current device (cached per device)
static int device_cus() {
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cache[dev] <= 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
      v = 256;
    cache[dev] = v;
  }
  return cache[dev];
}

// G = L_D^-1 by recursive doubling over the 64 x 64 diagonal inverses left by the panels:
// X21 = -X22 (L21 X11), two GEMMs per level, for nz problems in grid.z: problem z's L_D, G and
// scratch are the b x b blocks at D + z*zD, G + z*zG and S + z*zS (zn, step, zdiv: which
// problems take part, as in GemmArgs).  bta_invert_block reads block i's L_Di and G_i slots and
// the chain's scratch; it may run on another stream than the sweep once block i's panels are
// done.
static int invert_levels(double* D, long long zD, double* G, long long zG, double* S,
                         long long zS, int b, int nz, const int32_t* zn, int step, int zdiv,
                         int maxwg, hipStream_t s) {
  for (int sz = kPanel; sz < b; sz *= 2) {
    const int P = (b - sz + 2 * sz - 1) / (2 * sz);
    const int s2 = b - 2 * (P - 1) * sz - sz < sz ? b - 2 * (P - 1) * sz - sz : sz;
    const long long ystep = 2LL * sz * (b + 1);
    {  // T = L21 * X11  (X11 lower)
      GemmArgs g{};
      g.nph = 1;
      g.ph[0].A = view_plain(D + sz, b, zD);
      g.ph[0].B = view_plain(G, b, zG);
      g.ph[0].K = g.ph[0].Klast = sz;
      g.ph[0].kmode = KR_GE_N0;
      g.ph[0].triB = TRI_LOWER;
      g.ph[0].alpha = 1.0;
      view_set_y(g.ph[0].A, ystep);
      view_set_y(g.ph[0].B, ystep);
      g.C = view_plain(S + sz, b, zS);
      view_set_y(g.C, ystep);
      g.M = sz; g.Mlast = s2; g.N = g.Nlast = sz;
      g.beta = 0.0;
      g.omode = OUT_ALL;
      g.tag = GT_TRTRI;
      g.blk = b;
      g.maxwg = maxwg;
      g.zn = zn;
      g.step = step;
      g.zdiv = zdiv;
      if (launch_gemm(g, P, nz, s)) return ADELIA_E_HIP_INTERNAL;
    }
    {  // X21 = -X22 * T  (X22 lower)
      GemmArgs g{};
      g.nph = 1;
      g.ph[0].A = view_plain(G + sz + (long long)sz * b, b, zG);
      g.ph[0].B = view_plain(S + sz, b, zS);
      g.ph[0].K = sz; g.ph[0].Klast = s2;
      g.ph[0].kmode = KR_LT_M1;
      g.ph[0].triA = TRI_LOWER;
      g.ph[0].alpha = -1.0;
      view_set_y(g.ph[0].A, ystep);
      view_set_y(g.ph[0].B, ystep);
      g.C = view_plain(G + sz, b, zG);
      view_set_y(g.C, ystep);
      g.M = sz; g.Mlast = s2; g.N = g.Nlast = sz;
      g.beta = 0.0;
      g.omode = OUT_ALL;
      g.tag = GT_TRTRI;
      g.blk = b;
      g.maxwg = maxwg;
      g.zn = zn;
      g.step = step;
      g.zdiv = zdiv;
      if (launch_gemm(g, P, nz, s)) return ADELIA_E_HIP_INTERNAL;
    }
  }
  return 0;
}

int bta_invert_block(const BtaChains& c, int i, hipStream_t s) {
  const long long bb = (long long)c.b * c.b;
  return invert_levels(c.D + blk_off(i, c.slotsD, c.sD ? c.sD : bb), c.zD,
                       c.G + blk_off(i, c.slotsG, bb),
                       c.zG, c.scratch, c.zS, c.b, c.nz, c.zn, i, 0, c.inv_maxwg, s);
}

int bta_invert_blocks(double* D, long long sD, double* G, double* S, int b, int nzb, int zdiv,
                      const int32_t* zn, hipStream_t s) {
  const long long bb = (long long)b * b;
  return invert_levels(D, sD, G, bb, S, bb, b, nzb, zn, 0, zdiv, 0, s);
}

int bta_forward_block(const BtaChains& c, int i, hipStream_t s, const Lookahead* la) {
  const int b = c.b, ap = c.ap, n = c.n, nz = c.nz;
  const long long bb = (long long)b * b;
  const int ldT = b + ap;
  const int npanel = (b + kPanel - 1) / kPanel;
  const long long sD = c.sD ? c.sD : bb;
  double* Dblk = c.D + blk_off(i, c.slotsD, sD);
  double* Gblk = c.G + blk_off(i, c.slotsG, bb);
  double* LBC = c.LBC + blk_off(i, c.slotsLBC, (long long)ldT * b);
  const bool hasB = i < n - 1;
  // 0. the rows solved with the panels of L_Di: [B_i; C~_i] (C~_i alone for the last block)
  if (hasB && !c.b_in_place &&
      launch_copy2d(c.Bin + blk_off(i, c.slotsB, bb), b, c.zB, LBC, ldT, c.zLBC, b, b, nz, s))
    return ADELIA_E_HIP_INTERNAL;
  if (ap > 0 && !c.refactor &&
      launch_copy2d(c.C + (long long)i * ap * b, ap, c.zC, LBC + b, ldT, c.zLBC, ap, b, nz, s))
    return ADELIA_E_HIP_INTERNAL;
  double* Rows = hasB ? LBC : LBC + b;
  const int mT = (hasB ? b : 0) + (c.refactor ? 0 : ap);
  // rank-64 update of the columns from `from` on (the rows below them and the rows of
  // [B_i; C~_i]) with panel k
  auto trailing_args = [&](int k, int from) -> GemmArgs {
    const int c0 = k * kPanel;
    const int rest = b - from;
    GemmArgs g{};
    g.nph = 1;
    g.ph[0].A = view_rowsplit(Dblk + from + (long long)c0 * b, b, c.zD,
                              Rows + (long long)c0 * ldT, ldT, c.zLBC, rest);
    g.ph[0].B = view_plain(Dblk + from + (long long)c0 * b, b, c.zD, true);
    g.ph[0].K = g.ph[0].Klast = kPanel;
    g.ph[0].kmode = KR_FULL;
    g.ph[0].alpha = -1.0;
    g.C = view_rowsplit(Dblk + from + (long long)from * b, b, c.zD,
                        Rows + (long long)from * ldT, ldT, c.zLBC, rest);
    g.M = g.Mlast = rest + mT;
    g.N = g.Nlast = rest;
    g.beta = 1.0;
    g.omode = OUT_LOWER;  // lower for the block's own rows, every column of the rows below
    g.tag = GT_TRAIL;
    g.blk = c.b;
    g.zn = c.zn;
    g.step = i;
    return g;
  };
  // 1. blocked Cholesky of D_i; each panel also solves its columns of [B_i; C~_i] (the fused
  //    TRSM of Alg. 1, which with the rhs row yields z_i), and the trailing updates cover the
  //    block and those rows alike.  With the look-ahead, panel k applies panel k-1's update to
  //    its own columns, and the update of the columns from c0 + 64 on runs beside it: in the
  //    same launch (batches whose panel workgroups fit on the CUs: one step per launch, in
  //    stream order, with no cross-stream waits; four chains at b = 1024, 132 workgroups:
  //    22.9 against 23.7 ms per objective) or on the look-ahead stream.
  const bool fuse = la && 1LL * nz * panel_workgroups(b, 0, mT) <= la->cus;
  // Batches whose panel workgroups outnumber the CUs split each panel: one workgroup per chain
  // factors the diagonal tile, then one GEMM launch solves the panel's rows in place,
  // R = A L_kk^-T - P V^T with V = L_kk^-1 Q (P, Q: the previous panel's columns on the rows and
  // on the diagonal tile; that term is the look-ahead update (A - P Q^T) L_kk^-T), instead of
  // every row workgroup factoring the diagonal tile again.
  const int cus = la ? la->cus : device_cus();
  const bool split = !fuse && (long long)nz * panel_workgroups(b, 0, mT) > cus &&
                     (!la || c.Vp);
  auto panel = [&](int k, int upd) -> int {
    const int c0 = k * kPanel;
    double* ldp = c.ldpart + (long long)i * npanel + k;
    if (!split)
      return launch_potrf_panel(Dblk, c.zD, Gblk, c.zG, ldp, c.zLd, c.info, c.cnt, c.zn, i, b, c0,
                                (long long)i * b, mT ? Rows : nullptr, c.zLBC, ldT, mT, upd, nz,
                                s);
    const bool u = upd && c0 >= kPanel;
    if (launch_panel_diag(Dblk, c.zD, Gblk, c.zG, ldp, c.zLd, c.info, c.cnt, c.zn, i, b, c0,
                          (long long)i * b, u ? 1 : 0, u ? c.Vp : nullptr, c.zVp, nz, s))
      return -1;
    const int w = std::min(kPanel, b - c0);
    const int rest = b - c0 - w;
    if (rest + mT <= 0) return 0;
    GemmArgs g{};
    g.nph = u ? 2 : 1;
    g.ph[0].A = view_rowsplit(Dblk + c0 + w + (long long)c0 * b, b, c.zD,
                              Rows + (long long)c0 * ldT, ldT, c.zLBC, rest);
    g.ph[0].B = view_plain(Gblk + c0 + (long long)c0 * b, b, c.zG, true);
    g.ph[0].K = g.ph[0].Klast = w;
    g.ph[0].kmode = KR_LT_N1;
    g.ph[0].triB = TRI_UPPER;
    g.ph[0].alpha = 1.0;
    if (u) {
      g.ph[1].A = view_rowsplit(Dblk + c0 + w + (long long)(c0 - kPanel) * b, b, c.zD,
                                Rows + (long long)(c0 - kPanel) * ldT, ldT, c.zLBC, rest);
      g.ph[1].B = view_plain(c.Vp, kPanel, c.zVp, true);
      g.ph[1].K = g.ph[1].Klast = kPanel;
      g.ph[1].kmode = KR_FULL;
      g.ph[1].alpha = -1.0;
    }
    g.C = g.ph[0].A;  // in place: each tile reads its own rows of A before it stores them
    g.M = g.Mlast = rest + mT;
    g.N = g.Nlast = w;
    g.beta = 0.0;
    g.omode = OUT_ALL;
    g.tag = GT_PROWS;
    g.blk = c.b;
    g.zn = c.zn;
    g.step = i;
    return launch_gemm(g, 1, nz, s);
  };
  for (int k = 0; k < npanel; ++k) {
    const int c0 = k * kPanel;
    double* ldp = c.ldpart + (long long)i * npanel + k;
    if (fuse) {
      const bool upd = k >= 1 && b - (c0 + kPanel) > 0;
      const GemmArgs u = upd ? trailing_args(k - 1, c0 + kPanel) : GemmArgs{};
      if (launch_panel_step(Dblk, c.zD, Gblk, c.zG, ldp, c.zLd, c.info, c.cnt, c.zn, i, b, c0,
                            (long long)i * b, mT ? Rows : nullptr, c.zLBC, ldT, mT, 1, nz,
                            upd ? &u : nullptr, la->maxwg, s))
        return ADELIA_E_HIP_INTERNAL;
      if (la->mark && k == std::min(la->mark_step, npanel - 1) &&
          hipEventRecord(la->mark, s) != hipSuccess)
        return ADELIA_E_HIP_INTERNAL;
      continue;
    }
    // panel k waits for the update the look-ahead stream issued after panel k-2
    if (la && k >= 2 && hipStreamWaitEvent(s, la->tdone[(k - 2) % 3], 0) != hipSuccess)
      return ADELIA_E_HIP_INTERNAL;
    if (panel(k, la ? 1 : 0)) return ADELIA_E_HIP_INTERNAL;
    if (la && la->mark && k == std::min(la->mark_step, npanel - 1) &&
        hipEventRecord(la->mark, s) != hipSuccess)
      return ADELIA_E_HIP_INTERNAL;
    if (la) {
      // panel k+1 applies this panel's update to its own columns; the columns after it are
      // updated on the look-ahead stream
      if (b - c0 - 2 * kPanel > 0) {
        if (hipEventRecord(la->pdone[k % 3], s) != hipSuccess ||
            hipStreamWaitEvent(la->ts, la->pdone[k % 3], 0) != hipSuccess)
          return ADELIA_E_HIP_INTERNAL;
        const GemmArgs g = trailing_args(k, c0 + 2 * kPanel);
        if (launch_gemm(g, 1, nz, la->ts)) return ADELIA_E_HIP_INTERNAL;
        if (hipEventRecord(la->tdone[k % 3], la->ts) != hipSuccess) return ADELIA_E_HIP_INTERNAL;
      }
    } else if (b - c0 - kPanel > 0) {
      const GemmArgs g = trailing_args(k, c0 + kPanel);
      if (launch_gemm(g, 1, nz, s)) return ADELIA_E_HIP_INTERNAL;
    }
  }
  // 2. the full inverse, when the caller needs it inline
  if (c.invert) {
    const int r = bta_invert_block(c, i, s);
    if (r) return r;
  }
  // 3. Schur update of the next diagonal block, next arrow block and the tip (a rebuilt block
  //    has its successor's carry stored already)
  if (!c.refactor && (hasB || ap > 0)) {
    GemmArgs g{};
    g.nph = 1;
    g.ph[0].alpha = -1.0;
    g.ph[0].K = g.ph[0].Klast = b;
    g.ph[0].kmode = KR_FULL;
    g.beta = 1.0;
    g.omode = OUT_LOWER;
    g.ph[0].A = view_plain(Rows, ldT, c.zLBC);
    g.ph[0].B = view_plain(Rows, ldT, c.zLBC, true);
    if (hasB) {
      double* Dn = c.D + blk_off(i + 1, c.slotsD, sD);
      double* Cn = c.C + (long long)(i + 1) * ap * b;
      View v = view_plain(Dn, b, c.zD);
      v.rs = b; v.cs = b;
      v.p[1] = Cn; v.sr[1] = 1; v.sc[1] = ap; v.zs[1] = c.zC;
      v.p[3] = c.T; v.sr[3] = 1; v.sc[3] = ap; v.zs[3] = c.zT;
      g.C = v;
    } else {
      g.C = view_plain(c.T, ap, c.zT);
    }
    g.M = g.N = g.Mlast = g.Nlast = mT;
    g.tag = GT_SYRK;
    g.blk = c.b;
    g.zn = c.zn;
    g.step = i;
    g.tail = c.tail;
    if (launch_gemm(g, 1, nz, s)) return ADELIA_E_HIP_INTERNAL;
  }
  return 0;
}

int bta_tip(const BtaChains& c, hipStream_t s) {
  const int npanel = (c.b + kPanel - 1) / kPanel;
  if (c.ap == 0) {
    // no tip and no rhs row: an empty tip contributes log 1 = 0
    return launch_fill_strided(c.ldpart + (long long)c.n * npanel, c.zLd, c.nz, 0.0, s)
               ? ADELIA_E_HIP_INTERNAL : 0;
  }
  if (launch_tip(c.T, c.zT, c.a, c.ap, c.ldpart + (long long)c.n * npanel, c.zLd, c.info,
                 (long long)c.n * c.b, c.zsq, c.ZT, c.zZT, c.xT, c.zXT, c.nz, s))
    return ADELIA_E_HIP_INTERNAL;
  return 0;
}

int bta_forward(const BtaChains& c, hipStream_t s) {
  for (int i = 0; i < c.n; ++i) {
    int r = bta_forward_block(c, i, s);
    if (r) return r;
  }
  return bta_tip(c, s);
}

struct SelinvPtrs {
  const double* Gj;
  const double* LCj;
  const double* LBj;
  double *Wm, *V, *ZDj, *ZCj, *ZBj, *ZDn, *ZCn;
  bool last;
};

static SelinvPtrs selinv_ptrs(const SelinvChains& c, int j) {
  const int b = c.b, a = c.a, n = c.n;
  const long long bb = (long long)b * b;
  SelinvPtrs p;
  p.Gj = c.G + blk_off(j, c.slotsG, bb);
  p.LCj = c.LC + (long long)j * c.sLC;
  p.Wm = c.W + blk_off(j, c.slotsW, bb + (long long)a * b);
  p.V = p.Wm + bb;
  p.ZDj = c.ZD + blk_off(j, c.slotsZD, bb);
  p.ZCj = a ? c.ZC + blk_off(j, c.slotsZC, (long long)a * b) : nullptr;
  p.last = (j == n - 1);
  p.LBj = p.last ? nullptr : c.LB + blk_off(j, c.slotsLB, c.sLB);
  p.ZBj = p.last ? nullptr : c.ZB + blk_off(j, c.slotsZB, bb);
  p.ZDn = p.last ? nullptr : c.ZD + blk_off(j + 1, c.slotsZD, bb);
  p.ZCn = (p.last || !a) ? nullptr : c.ZC + blk_off(j + 1, c.slotsZC, (long long)a * b);
  return p;
}

int selinv_prepare(const SelinvChains& c, int j, hipStream_t s) {
  const int b = c.b, a = c.a, nz = c.nz;
  const SelinvPtrs p = selinv_ptrs(c, j);
  const long long zW = c.zW;
  // S1: [W; V] = [L_Bj; L_Cj] G_j
  {
    GemmArgs g{};
    g.nph = 1;
    if (!p.last && !c.w_external) {
      g.ph[0].A = view_rowsplit(const_cast<double*>(p.LBj), c.ldLB, c.zLB,
                                const_cast<double*>(p.LCj), c.ldLC, c.zLC, b);
      g.C = view_rowsplit(p.Wm, b, zW, p.V, a ? a : 1, zW, b);
      g.M = g.Mlast = b + a;
    } else {
      g.ph[0].A = view_plain(const_cast<double*>(p.LCj), c.ldLC, c.zLC);
      g.C = view_plain(p.V, a ? a : 1, zW);
      g.M = g.Mlast = a;
    }
    g.ph[0].B = view_plain(const_cast<double*>(p.Gj), b, c.zG);
    g.ph[0].K = g.ph[0].Klast = b;
    g.ph[0].kmode = KR_GE_N0;
    g.ph[0].triB = TRI_LOWER;
    g.ph[0].alpha = 1.0;
    g.N = g.Nlast = b;
    g.beta = 0.0;
    g.omode = OUT_ALL;
    g.tag = GT_SI_W;
    g.blk = c.b;
    g.maxwg = c.prep_maxwg;
    g.zn = c.zn;
    g.step = j;
    if (g.M > 0 && launch_gemm(g, 1, nz, s)) return ADELIA_E_HIP_INTERNAL;
  }
  // S3 (first term): lower triangle of Z_Dj = G_j^T G_j
  {
    GemmArgs g{};
    g.nph = 1;
    g.ph[0].A = view_plain(const_cast<double*>(p.Gj), b, c.zG, true);
    g.ph[0].B = view_plain(const_cast<double*>(p.Gj), b, c.zG);
    g.ph[0].K = g.ph[0].Klast = b;
    g.ph[0].kmode = KR_GE_MAX;
    g.ph[0].triA = TRI_UPPER;
    g.ph[0].triB = TRI_LOWER;
    g.ph[0].alpha = 1.0;
    g.C = view_plain(p.ZDj, b, c.zZD);
    g.M = g.N = g.Mlast = g.Nlast = b;
    g.beta = 0.0;
    g.omode = c.w_external ? OUT_LOWER_MIRROR : OUT_LOWER;  // W_j reads its full columns
    g.tag = GT_SI_D;
    g.blk = c.b;
    g.maxwg = c.prep_maxwg;
    g.zn = c.zn;
    g.step = j;
    if (launch_gemm(g, 1, nz, s)) return ADELIA_E_HIP_INTERNAL;
  }
  return 0;
}

int selinv_finish(const SelinvChains& c, int j, hipStream_t s) {
  const int b = c.b, a = c.a, nz = c.nz;
  const SelinvPtrs p = selinv_ptrs(c, j);
  const long long zW = c.zW;
  // S2: [Z_Bj; Z_Cj] = -Zhat_{j+1} [W; V]
  if (!p.last) {
    GemmArgs g{};
    g.nph = 1;
    View A = view_plain(p.ZDn, b, c.zZD);
    A.rs = b; A.cs = b;
    if (a) {
      A.p[1] = p.ZCn; A.sr[1] = 1; A.sc[1] = a; A.zs[1] = c.zZC;          // Z_C(r-b, c)
      A.p[2] = p.ZCn; A.sr[2] = a; A.sc[2] = 1; A.zs[2] = c.zZC;          // Z_C^T
      A.p[3] = const_cast<double*>(c.ZT); A.sr[3] = 1; A.sc[3] = a; A.zs[3] = c.zZT;
    }
    g.ph[0].A = A;
    g.ph[0].B = view_rowsplit(p.Wm, b, zW, p.V, a ? a : 1, zW, b);
    g.ph[0].K = g.ph[0].Klast = b + a;
    g.ph[0].kmode = KR_FULL;
    g.ph[0].alpha = -1.0;
    g.C = view_rowsplit(p.ZBj, b, c.zZB, p.ZCj ? p.ZCj : p.ZBj, a ? a : 1, c.zZC, b);
    // a few arrow rows would add a row of mostly empty 64-row tiles to the product (a second
    // round of workgroups when the tiles exactly fill the device): they go through the short
    // product kernel instead
    const bool skinny = a > 0 && a <= kSkinnyRows;
    g.M = g.Mlast = skinny ? b : b + a;
    g.N = g.Nlast = b;
    g.beta = 0.0;
    g.omode = OUT_ALL;
    g.tag = GT_SI_Z;
    g.blk = c.b;
    g.maxwg = c.fin_maxwg;
    g.zn = c.zn;
    g.step = j;
    g.tail = c.tail;
    if (launch_gemm(g, 1, nz, s)) return ADELIA_E_HIP_INTERNAL;
    if (skinny) {  // Z_Cj = -(Z_C,j+1 W + Z_T V)
      Skinny k{};
      k.m = a; k.N = b; k.K1 = b; k.K2 = a;
      k.A1 = p.ZCn; k.lda1 = a; k.zA1 = c.zZC;
      k.B1 = p.Wm; k.ldb1 = b; k.zB1 = zW;
      k.A2 = c.ZT; k.lda2 = a; k.zA2 = c.zZT;
      k.B2 = p.V; k.ldb2 = a; k.zB2 = zW;
      k.C = p.ZCj; k.ldc = a; k.zC = c.zZC;
      k.alpha = -1.0; k.beta = 0.0;
      k.zn = c.zn; k.step = j;
      if (launch_skinny(k, nz, s)) return ADELIA_E_HIP_INTERNAL;
    }
  } else if (a) {
    GemmArgs g{};
    g.nph = 1;
    g.ph[0].A = view_plain(const_cast<double*>(c.ZT), a, c.zZT);
    g.ph[0].B = view_plain(p.V, a, zW);
    g.ph[0].K = g.ph[0].Klast = a;
    g.ph[0].kmode = KR_FULL;
    g.ph[0].alpha = -1.0;
    g.C = view_plain(p.ZCj, a, c.zZC);
    g.M = g.Mlast = a;
    g.N = g.Nlast = b;
    g.beta = 0.0;
    g.omode = OUT_ALL;
    g.tag = GT_SI_Z;
    g.blk = c.b;
    g.maxwg = c.fin_maxwg;
    g.zn = c.zn;
    g.step = j;
    if (launch_gemm(g, 1, nz, s)) return ADELIA_E_HIP_INTERNAL;
  }
  // S3: Z_Dj -= [Z_Bj; Z_Cj]^T [W; V] on the lower triangle holding G^T G, mirrored to a full
  // symmetric block (the mirror is written even when there is nothing to subtract)
  {
    GemmArgs g{};
    g.nph = 1;
    if (!p.last) {
      g.ph[0].A = view_rowsplit(p.ZBj, b, c.zZB, p.ZCj ? p.ZCj : p.ZBj, a ? a : 1, c.zZC, b, true);
      g.ph[0].B = view_rowsplit(p.Wm, b, zW, p.V, a ? a : 1, zW, b);
      g.ph[0].K = g.ph[0].Klast = b + a;
    } else {
      g.ph[0].A = view_plain(p.ZCj ? p.ZCj : p.ZDj, a ? a : 1, c.zZC, true);
      g.ph[0].B = view_plain(p.V, a ? a : 1, zW);
      g.ph[0].K = g.ph[0].Klast = a;  // 0 when there is no arrow: only the mirror is written
    }
    g.ph[0].kmode = KR_FULL;
    g.ph[0].alpha = -1.0;
    g.C = view_plain(p.ZDj, b, c.zZD);
    g.M = g.N = g.Mlast = g.Nlast = b;
    g.beta = 1.0;
    g.omode = OUT_LOWER_MIRROR;
    g.tag = GT_SI_D;
    g.blk = c.b;
    g.maxwg = c.fin_maxwg;
    g.zn = c.zn;
    g.step = j;
    g.tail = c.tail;
    if (launch_gemm(g, 1, nz, s)) return ADELIA_E_HIP_INTERNAL;
  }
  return 0;
}

int bta_upper_solve(const SolveChains& c, hipStream_t s) {
  for (int i = c.n - 1; i >= 0; --i)
    if (bta_upper_solve_block(c, i, s)) return ADELIA_E_HIP_INTERNAL;
  return bta_upper_solve_tip(c, s);
}

int bta_upper_solve_block(const SolveChains& c, int i, hipStream_t s) {
  const int b = c.b, a = c.a, n = c.n, nz = c.nz;
  const long long bb = (long long)b * b;
  {
    const double* LCi = c.LC + (long long)i * c.sLC;
    GemvT g{};
    if (i < n - 1) {
      g.A = c.LB + blk_off(i, c.slotsLB, c.sLB); g.ld = c.ldLB; g.zA = c.zLB;
      g.x = c.x + (long long)(i + 1) * b; g.zx = c.zx; g.incx = 1;
      g.alpha = -1.0;
    }
    if (a) {
      g.A2 = LCi; g.ld2 = c.ldLC; g.zA2 = c.zLC; g.r2 = a;
      g.x2 = c.xT; g.zx2 = c.zxT;
      g.alpha2 = -1.0;
    }
    g.y0 = c.z + (long long)i * c.sz_blk; g.zy0 = c.zz; g.incy0 = c.sz_elem;
    g.beta = 1.0;
    g.y = c.y; g.zy = c.zy; g.incy = 1;
    g.M = b; g.K = b; g.lowerA = 0;
    g.zn = c.zn; g.step = i; g.zn_stride = c.zn_stride;
    if (launch_gemv_t(g, nz, s)) return ADELIA_E_HIP_INTERNAL;
    GemvT h{};
    h.A = c.G + blk_off(i, c.slotsG, bb); h.ld = b; h.zA = c.zG;
    h.x = c.y; h.zx = c.zy; h.incx = 1;
    h.alpha = 1.0;
    h.y = c.x + (long long)i * b; h.zy = c.zx; h.incy = 1;
    h.M = b; h.K = b; h.lowerA = 1;
    h.zn = c.zn; h.step = i; h.zn_stride = c.zn_stride;
    if (launch_gemv_t(h, nz, s)) return ADELIA_E_HIP_INTERNAL;
  }
  return 0;
}

int bta_upper_solve_tip(const SolveChains& c, hipStream_t s) {
  const int b = c.b, a = c.a, n = c.n, nz = c.nz;
  // the tip part of x
  if (a && c.xT) {
    if (launch_copy2d(c.xT, a, c.zxT, c.x + (long long)n * b, a, c.zx, a, 1, nz, s))
      return ADELIA_E_HIP_INTERNAL;
  }
  return 0;
}

}  // namespace adelia
