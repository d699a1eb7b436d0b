// INLA entry points: model set-up (validation, integer index structures, upload), workspace
// layout and the orchestration of one objective / gradient evaluation (Sec. III-A, Eq. 5).
//
// Chains: for theta point p, chain 2p is the conditional precision Qc (BTA, arrow = fixed
// effects plus the right-hand-side row) and chain 2p+1 the prior Qp (its arrow blocks are zero
// and its tip is tip_prec * I), so both run through the same batched launches.
#include "../../include/adelia.h"
#include "common.h"
#include "inla_dev.h"
#include "internal_api.h"
#include "launchers.h"
#include "profile.h"

#include <algorithm>
#include <climits>
#include <cstring>
#include <map>
#include <string>
#include <vector>

using namespace adelia;

// A second stream per model forms the block inverses L_Di^-1 of a gradient's forward sweep
// while the sweep goes on with the next blocks (the inverses are needed only by the backward
// pass).  Events order it against the caller's stream; the ring of three D slots in gradient
// workspaces gives each inversion one block step of slack.
struct SideRes {
  hipStream_t s2;
  hipEvent_t ready[3], done[3];
  Lookahead la;  // look-ahead of the sweep: fused steps, or its own stream for large batches
  int side_maxwg;  // workgroup cap of the launches on s2
};

struct inla_model_s {
  int device;
  int param;
  ModelDev M;
  const ModelDev* Md;  // device copy of M (inside dev_mem), read by the kernels
  void* dev_mem;
  SideRes side;
  bool has_side;
  // the workspace holding the factors of the last inla_objective(SAVE_FACTORS): one
  // inla_grad(REUSE_FACTORS) on it consumes them (the reverse pass overwrites G^T G with Z_D);
  // any other call on that workspace discards them
  const void* saved_ws;
  // Two-sided split (ADELIA_SPLIT; the two-phase decomposition of Sec. III-C with P = 2 on one
  // GPU): half A = blocks 0..sep, half B = blocks n-1..sep in reverse order, each a model of its
  // own (B's separator block and fixed-effect prior are zero, its hyperparameter prior absent),
  // swept in the same launches toward the separator block; the separator and the tip form the
  // reduced system.  split_sep < 0: not available (n < 3).
  int split_sep;
  inla_model half[2];
  ModelDev* half_dev;   // device: the two halves' descriptions, A then B
  int32_t* zn_split;    // device: blocks swept per half chain [A, A, B, B]
  ModelDev Mh;          // layout of the halves (the longer half)
  ModelDev Mr;          // layout of the reduced system (one block)
};

namespace {

// What one evaluation runs on: the host description that sizes the workspace and the launches
// (for an uneven batch, the largest instance of a group), the model(s) the kernels read, and for
// an uneven batch the block count of every chain (its sweeps skip the steps past it).
struct Eval {
  const ModelDev& M;
  Models dev;
  const int32_t* zn;
};

struct InlaWs {
  int batch, nz, n, b, a, ap, k, d, npanel;
  bool grad;
  // carry-only gradient: the forward keeps each block's Schur-updated diagonal block (Dc) and
  // its arrow rows [L_C | z] (LCz, ld ap) instead of the factors; the backward rebuilds
  // L_D, L_B, G, W and G^T G block by block in small rings
  bool carry;
  // stored-factor gradient: every block's L_D is kept as well, and the Z-independent part of the
  // selected inversion (G, [W; V], G^T G) is formed for all blocks in one pass after the sweep
  bool defer;
  double *Dc, *LCz;
  long long zDc, zLCz;
  int slotsW, slotsZD;
  int slotsD, slotsB, slotsLBC, slotsG;
  double *D, *Bin, *LBC, *G, *C, *T, *S, *ldpart, *ld, *zsq, *ZT, *xT;
  long long zD, zB, zLBC, zG, zC, zT, zS, zLd, zZT, zXT;
  long long sD;  // slot stride of D
  int32_t* info;
  int32_t* cnt;   // panel write-back counters (nz), zero between launches
  double *phi, *dphi, *tau;
  double *Th, *fv;
  int32_t* finfo;
  long long zq, zr;  // per-point strides of qD/qB and resid
  double* gv;
  double* Vp;
  long long zVp;
  double *x, *y, *W, *ZD, *ZB, *ZC, *TD, *TB, *O, *qD, *qB, *resid;
  long long zx, zy, zW, zZD, zZB, zZC, zTr, zO;
  double* tws;  // kTailTiles partial tiles: the K split of the main stream's long products
  size_t bytes;
};

InlaWs layout(const ModelDev& M, int batch, bool grad, char* base, bool carry = false) {
  InlaWs w{};
  w.batch = batch;
  w.carry = grad && carry;
  w.nz = 2 * batch;
  w.n = M.nt; w.b = M.b; w.a = M.a; w.ap = M.a + 1; w.k = M.k; w.d = M.d;
  w.npanel = (M.b + kPanel - 1) / kPanel;
  w.grad = grad;
  const long long bb = (long long)M.b * M.b;
  const int n = M.nt;
  const bool stored = grad && !w.carry;  // every block's factor kept
  w.defer = stored;
  // carry-only: rings of three blocks for the pipelined reverse pass; an objective: three D
  // slots and two [L_B; L_C] slots, so that D_{i+2} and B_{i+1} can be assembled while block
  // i is factored (D_{i-1} and [L_B; L_C]_{i-1} are no longer read by then)
  w.slotsD = stored ? n : 3;
  w.slotsB = 1;
  w.slotsLBC = stored ? n : (w.carry ? 3 : 2);
  w.slotsG = stored ? n : (w.carry ? 3 : 1);
  w.slotsW = stored ? n : 3;
  w.slotsZD = stored ? n : 3;
  size_t off = 0;
  auto take = [&](long long per_chain, int chains, long long& stride) {
    stride = per_chain;
    double* p = base ? reinterpret_cast<double*>(base + off) : nullptr;
    off = align_up(off + (size_t)per_chain * chains * sizeof(double));
    return p;
  };
  long long dummy;
  // finite-difference stencil scratch first: its place does not depend on the batch size.  It
  // holds the largest stencil (the 2d^2 + 1 points of the FD Hessian) and the 2d + 1 gradients
  // of the Hessian of Eq. 12.
  const int npts = 2 * M.d * M.d + 1;
  w.Th = take((long long)npts * M.d, 1, dummy);
  w.fv = take(npts, 1, dummy);
  w.gv = take((long long)(2 * M.d + 1) * M.d, 1, dummy);
  {
    double* p = base ? reinterpret_cast<double*>(base + off) : nullptr;
    w.finfo = reinterpret_cast<int32_t*>(p);
    off = align_up(off + (size_t)npts * sizeof(int32_t));
  }
  const int nz = w.nz;
  // a stored-factor gradient factors D_t in the slot of [W_t; V_t] (b^2 + a b doubles), free
  // until the side work has read L_Dt; the other modes keep a ring of b x b slots
  w.sD = bb;
  if (!stored) w.D = take(w.slotsD * bb, nz, w.zD);
  w.Bin = take(w.slotsB * bb, nz, w.zB);
  w.LBC = take((long long)w.slotsLBC * (M.b + w.ap) * M.b, nz, w.zLBC);
  w.G = take(w.slotsG * bb, nz, w.zG);
  w.C = take((long long)n * w.ap * M.b, nz, w.zC);
  w.T = take((long long)w.ap * w.ap, nz, w.zT);
  w.S = take(bb, nz, w.zS);
  w.ldpart = take((long long)n * w.npanel + 1, nz, w.zLd);
  w.ld = take(1, nz, dummy);
  w.zsq = take(1, nz, dummy);
  w.ZT = take(std::max(1, w.a * w.a), nz, w.zZT);
  w.xT = take(std::max(1, w.a), nz, w.zXT);
  w.Vp = take((long long)kPanel * kPanel, nz, w.zVp);
  {
    double* p = base ? reinterpret_cast<double*>(base + off) : nullptr;
    w.info = reinterpret_cast<int32_t*>(p);
    w.cnt = w.info ? w.info + nz : nullptr;
    off = align_up(off + (size_t)2 * nz * sizeof(int32_t));
  }
  w.tws = take((long long)kTailTiles * 64 * 64, 1, dummy);
  const long long NE = 9LL * M.k * M.k;
  w.phi = take(NE, batch, dummy);
  w.dphi = take(NE * M.d, batch, dummy);
  w.tau = take(M.k, batch, dummy);
  if (grad) {
    const long long Nlat = (long long)n * M.b + M.a;
    w.x = take(Nlat, nz, w.zx);
    w.y = take(M.b, nz, w.zy);
    // [W_t; V_t] and G_t^T G_t (the Z-independent parts of the selected inversion) are formed
    // during the forward sweep, so they get a slot per block
    w.W = take((long long)w.slotsW * (bb + (long long)M.a * M.b), nz, w.zW);
    if (stored) {
      w.D = w.W;
      w.zD = w.zW;
      w.sD = bb + (long long)M.a * M.b;
    }
    w.ZD = take((long long)w.slotsZD * bb, nz, w.zZD);
    if (w.carry) {
      w.Dc = take((long long)n * bb, nz, w.zDc);
      w.LCz = take(std::max(1LL, (long long)n * w.ap * M.b), nz, w.zLCz);
    }
    w.ZB = take(bb, nz, w.zZB);
    w.ZC = take(std::max(1LL, 2LL * M.a * M.b), nz, w.zZC);
    w.TD = take((long long)n * 3 * M.k * M.k * M.nch_rows, nz, w.zTr);
    w.TB = take((long long)n * 3 * M.k * M.k * M.nch_rows, nz, dummy);
    w.O = take((long long)n * M.k * M.nch_obs, nz, w.zO);
    w.qD = take((long long)n * 3 * M.k * M.k, batch, w.zq);
    w.qB = take((long long)n * 3 * M.k * M.k, batch, dummy);
    w.resid = take((long long)M.k * M.nch_resid, batch, w.zr);
  }
  w.bytes = off + 256;
  return w;
}

BtaChains chains_of(const InlaWs& w) {
  BtaChains c{};
  c.n = w.n; c.b = w.b; c.a = w.a; c.ap = w.ap; c.nz = w.nz;
  c.D = w.D; c.zD = w.zD; c.slotsD = w.slotsD; c.sD = w.sD;
  c.Bin = w.Bin; c.zB = w.zB; c.slotsB = w.slotsB;
  c.C = w.C; c.zC = w.zC;
  c.LBC = w.LBC; c.zLBC = w.zLBC; c.slotsLBC = w.slotsLBC;
  c.invert = w.grad && !w.carry;
  c.T = w.T; c.zT = w.zT;
  c.G = w.G; c.zG = w.zG; c.slotsG = w.slotsG;
  c.ldpart = w.ldpart; c.zLd = w.zLd;
  c.info = w.info;
  c.cnt = w.cnt;
  c.scratch = w.S; c.zS = w.zS;
  c.zsq = w.zsq;
  if (w.grad && w.a > 0) {
    c.ZT = w.ZT; c.zZT = w.zZT;
    c.xT = w.xT; c.zXT = w.zXT;
  }
  c.Vp = w.Vp; c.zVp = w.zVp;
  return c;
}

#define LAUNCH_OK() (hipGetLastError() == hipSuccess)

// The selected-inversion view of the workspace (factors, [W; V] and Z blocks per chain).
SelinvChains selinv_of(const InlaWs& w) {
  const int b = w.b, ap = w.ap;
  const long long sLBC = (long long)(b + ap) * b;
  SelinvChains si{};
  si.n = w.n; si.b = b; si.a = w.a; si.nz = w.nz;
  si.G = w.G; si.zG = w.zG; si.slotsG = w.slotsG;
  si.LB = w.LBC; si.zLB = w.zLBC; si.slotsLB = w.slotsLBC; si.ldLB = b + ap; si.sLB = sLBC;
  si.LC = w.LBC + b; si.zLC = w.zLBC; si.ldLC = b + ap; si.sLC = sLBC;
  si.ZT = w.ZT; si.zZT = w.zZT;
  si.ZD = w.ZD; si.zZD = w.zZD; si.slotsZD = w.slotsZD;
  si.ZB = w.ZB; si.zZB = w.zZB; si.slotsZB = 1;
  si.ZC = w.ZC; si.zZC = w.zZC; si.slotsZC = 2;
  si.W = w.W; si.zW = w.zW; si.slotsW = w.slotsW;
  if (w.carry) {  // the arrow rows of every block, ld ap
    si.LC = w.LCz; si.zLC = w.zLCz; si.ldLC = ap; si.sLC = (long long)ap * b;
  }
  return si;
}

// The Z-independent part of the selected inversion of block j: V_j, G_j^T G_j and then
// W_j = L_Bj G_j = B_j (L_Dj L_Dj^T)^-1 = B_j G_j^T G_j from the sparse B_j (the dense product
// [L_Bj; L_Cj] G_j would cost b^3 flops per block), when a column of G_j^T G_j fits in LDS.
// The W_j product is bound by reading G_j^T G_j and writing W_j; about 512 workgroups over all
// chains keep HBM busy without crowding the work that runs beside it.
constexpr int kWGroups = 512;

// Columns of Y per LDS pass of the banded W_t kernel (0: the pattern does not suit it).
static int w_band_cols(const ModelDev& M) {
  if (!M.wband || M.wdeg > kWDeg || M.k < 1 || M.k > kMaxFields) return 0;
  const long long per = (long long)M.k * M.wband_w * (long long)sizeof(double);
  return (int)std::min<long long>(16, kWPassBytes / per);
}

// Columns of Y per pass of the LDS-batched W_t kernel (0: a column does not fit in 64 KB).
static int w_gtg_cols(int b) {
  return std::min<int>(kWBatch, (int)((64 * 1024) / ((size_t)b * sizeof(double))));
}

// W_t = B_t Y for nzl problems in grid.z (zdiv == 0: block t of each chain; zdiv > 0: the
// (chain, block) pairs of prepare_all), Y = G_t^T G_t stored in full: the banded kernel when the
// pattern suits it, else the LDS-batched one.
static int launch_w(const ModelDev& M, Models dev, int t, int zdiv, const int32_t* zn,
                    const double* Y, long long zY, double* W, long long zW, const double* phi,
                    int nzl, hipStream_t s) {
  const int b = M.b;
  const long long bb = (long long)b * b;
  const ProfToken tok = prof_begin(s);
  if (const int cb = w_band_cols(M)) {
    const int tiles = (M.ns + kWRows - 1) / kWRows;
    // about 2048 workgroups in all, each slice a whole number of LDS passes
    const int want = (int)std::max<long long>(1, 2048 / ((long long)nzl * tiles));
    const int passes = (b + cb - 1) / cb;
    const int slices0 = std::min(want, passes);
    const int cs = ((passes + slices0 - 1) / slices0) * cb;
    const int slices = (b + cs - 1) / cs;
    const dim3 grid(tiles, slices, nzl);
    const size_t lds = (size_t)M.k * cb * M.wband_w * sizeof(double);
    switch (M.k) {
      case 1: hipLaunchKernelGGL(w_band_kernel<1>, grid, dim3(256), lds, s, dev, t, zdiv, zn, Y, zY, W, zW, phi, cb, cs); break;
      case 2: hipLaunchKernelGGL(w_band_kernel<2>, grid, dim3(256), lds, s, dev, t, zdiv, zn, Y, zY, W, zW, phi, cb, cs); break;
      case 3: hipLaunchKernelGGL(w_band_kernel<3>, grid, dim3(256), lds, s, dev, t, zdiv, zn, Y, zY, W, zW, phi, cb, cs); break;
      default: hipLaunchKernelGGL(w_band_kernel<4>, grid, dim3(256), lds, s, dev, t, zdiv, zn, Y, zY, W, zW, phi, cb, cs); break;
    }
  } else {
    const int cg = w_gtg_cols(b);
    if (cg < 1) return ADELIA_E_HIP_INTERNAL;
    const int wg = std::max(1, std::min((b + cg - 1) / cg, kWGroups / nzl));
    hipLaunchKernelGGL(w_from_gtg_kernel, dim3(wg, 1, nzl), dim3(256),
                       (size_t)cg * b * sizeof(double), s, dev, t, zdiv, zn, Y, zY, W, zW, phi,
                       cg);
  }
  if (tok.valid)  // G^T G read and W written once per problem
    prof_end(tok, s, PK_WSPARSE, 0.0, 16.0 * nzl * (double)bb);
  return hipGetLastError() == hipSuccess ? 0 : ADELIA_E_HIP;
}

// Whether W_t can be formed from G_t^T G_t (else the dense product [L_B; L_C] G).
static bool w_sparse_ok(const ModelDev& M) { return w_band_cols(M) > 0 || w_gtg_cols(M.b) > 0; }

int prepare_block(const Eval& E, const InlaWs& w, SelinvChains si, int j, hipStream_t s) {
  const int b = w.b;
  const bool sparse_w = j < w.n - 1 && w_sparse_ok(E.M);
  si.w_external = sparse_w;
  if (selinv_prepare(si, j, s)) return ADELIA_E_HIP;
  if (sparse_w) {
    const long long bb = (long long)b * b;
    const double* Y = w.ZD + (long long)(j % w.slotsZD) * bb;
    double* Wm = w.W + (long long)(j % w.slotsW) * (bb + (long long)w.a * b);
    // chains past their block count skip the step: for the halves of the split their slot j
    // holds the separator's diagonal block
    return launch_w(E.M, E.dev, j, 0, E.zn, Y, w.zZD, Wm, w.zW, w.phi, w.nz, s);
  }
  return 0;
}

// The Z-independent part of the selected inversion of every block of every chain, once the
// sweep has left all factors in place (a stored-factor gradient): G_j = L_Dj^-1 by recursive
// doubling (block j's Z_D slot is its scratch), V_j = L_Cj G_j, G_j^T G_j in Z_Dj (mirrored to
// a full block for the W_j product) and W_j = B_j G_j^T G_j.  Each launch covers every (chain,
// block) pair in grid.z, z = chain * n + block, which the workspace's consecutive per-block
// slots make one stride; the chains go in groups that keep grid.z within its limit.
int prepare_all(const Eval& E, const InlaWs& w, hipStream_t s) {
  const int n = w.n, b = w.b, a = w.a, ap = w.ap;
  if (!w.defer || w.slotsD != n || w.slotsG != n || w.slotsLBC != n || w.slotsW != n ||
      w.slotsZD != n || w.zD != (long long)n * w.sD)
    return ADELIA_E_HIP_INTERNAL;
  const long long bb = (long long)b * b;
  const long long sLBC = (long long)(b + ap) * b;
  const long long sW = bb + (long long)a * b;
  const bool sparse_w = w_sparse_ok(E.M);
  const int per = std::max(2, (65535 / n) & ~1);  // whole points (two chains each)
  const long long sphi = 9LL * w.k * w.k;
  for (int c0 = 0; c0 < w.nz; c0 += per) {
    const int nzb = std::min(per, w.nz - c0) * n;
    const int32_t* zn = E.zn ? E.zn + c0 : nullptr;
    double* D = w.D + c0 * w.zD;
    double* G = w.G + c0 * w.zG;
    double* ZD = w.ZD + c0 * w.zZD;
    double* LC = w.LBC + c0 * w.zLBC + b;
    double* Wm = w.W + c0 * w.zW;
    if (bta_invert_blocks(D, w.sD, G, ZD, b, nzb, n, zn, s)) return ADELIA_E_HIP;
    if (!sparse_w) {
      // W_j cannot be formed from G_j^T G_j: the per-block dense products of the sweep's own
      // preparation
      SelinvChains si = selinv_of(w);
      si.zn = E.zn;
      if (c0 == 0)
        for (int j = 0; j < n; ++j)
          if (selinv_prepare(si, j, s)) return ADELIA_E_HIP;
      continue;
    }
    if (a > 0 && a <= kSkinnyRows) {  // V_j: a rows, G_j lower triangular
      Skinny k{};
      k.m = a; k.N = b; k.K1 = b; k.K2 = 0;
      k.A1 = LC; k.lda1 = b + ap; k.zA1 = sLBC;
      k.B1 = G; k.ldb1 = b; k.zB1 = bb;
      k.C = Wm + bb; k.ldc = a; k.zC = sW;
      k.alpha = 1.0; k.beta = 0.0;
      k.zn = zn; k.zdiv = n; k.lowerB = 1;
      if (launch_skinny(k, nzb, s)) return ADELIA_E_HIP;
    } else if (a > 0) {
      GemmArgs g{};
      g.nph = 1;
      g.ph[0].A = view_plain(LC, b + ap, sLBC);
      g.ph[0].B = view_plain(G, b, bb);
      g.ph[0].K = g.ph[0].Klast = b;
      g.ph[0].kmode = KR_GE_N0;
      g.ph[0].triB = TRI_LOWER;
      g.ph[0].alpha = 1.0;
      g.C = view_plain(Wm + bb, a, sW);
      g.M = g.Mlast = a;
      g.N = g.Nlast = b;
      g.beta = 0.0;
      g.omode = OUT_ALL;
      g.tag = GT_SI_W;
      g.blk = b;
      g.zn = zn;
      g.zdiv = n;
      if (launch_gemm(g, 1, nzb, s)) return ADELIA_E_HIP;
    }
    {  // G_j^T G_j, full (the W_j product reads whole columns)
      GemmArgs g{};
      g.nph = 1;
      g.ph[0].A = view_plain(G, b, bb, true);
      g.ph[0].B = view_plain(G, b, bb);
      g.ph[0].K = g.ph[0].Klast = b;
      g.ph[0].kmode = KR_GE_MAX;
      g.ph[0].triA = TRI_UPPER;
      g.ph[0].triB = TRI_LOWER;
      g.ph[0].alpha = 1.0;
      g.C = view_plain(ZD, b, bb);
      g.M = g.N = g.Mlast = g.Nlast = b;
      g.beta = 0.0;
      g.omode = OUT_LOWER_MIRROR;
      g.tag = GT_SI_D;
      g.blk = b;
      g.zn = zn;
      g.zdiv = n;
      if (launch_gemm(g, 1, nzb, s)) return ADELIA_E_HIP;
    }
    // W_j = B_j G_j^T G_j
    Models dev = E.dev;
    if (dev.each) dev.v += c0 / 2;
    if (launch_w(E.M, dev, 0, n, zn, ZD, bb, Wm, sW, w.phi + (c0 / 2) * sphi, nzb, s))
      return ADELIA_E_HIP;
  }
  return 0;
}

// Whether a stored-factor gradient forms its side work (G_j, [W_j; V_j], G_j^T G_j) block by
// block on the side stream beside the sweep rather than for all blocks after it: when the
// panel workgroups of a step fill at most half the CUs, the products have room beside them
// (b = 1024, one gradient: 44.5 against 47.0 ms); with more chains the side stream's tiles hold
// the CUs the next panel launch needs (four chains: 37.5 ms deferred against 40.0).
static bool side_beside_sweep(const InlaWs& w, const SideRes* side) {
  return side && 2LL * w.nz * panel_workgroups(w.b, 0, w.b + w.ap) <= side->la.cus;
}

// Assembly plus the forward sweeps of Qc and Qp for every theta point of the batch.
// tip == false (the halves of the two-sided split): the tips keep their Schur-complemented
// values, unfactored, for the reduced system.  A stored-factor gradient forms the
// Z-independent part of the selected inversion after the sweep (prepare_all) unless prep is
// false (the caller runs it).
int run_forward(const Eval& E, const InlaWs& w, const double* theta, hipStream_t s,
                const SideRes* side, bool tip = true, bool prep = true) {
  const ModelDev& M = E.M;
  const int nz = w.nz, n = w.n, b = w.b;
  hipLaunchKernelGGL(param_kernel, dim3(w.batch), dim3(256), 0, s, E.dev, theta, w.phi, w.dphi,
                     w.tau);
  if (!LAUNCH_OK()) return ADELIA_E_HIP;
  if (launch_fill_i32(w.info, nz, INT32_MAX, s)) return ADELIA_E_HIP;
  if (launch_fill_i32(w.cnt, nz, 0, s)) return ADELIA_E_HIP;
  const long long nb = (long long)n * b;
  hipLaunchKernelGGL(assemble_arrow_kernel, dim3((unsigned)((nb + 255) / 256), 1, nz), dim3(256),
                     0, s, E.dev, w.C, w.zC, nb, w.ap, w.tau);
  hipLaunchKernelGGL(assemble_tip_kernel, dim3(w.ap * w.ap, 1, nz), dim3(256), 0, s, E.dev, w.T,
                     w.zT, w.ap, w.tau);
  if (!LAUNCH_OK()) return ADELIA_E_HIP;
  const long long bb = (long long)b * b;
  const dim3 agrid(b, 1, nz);
  BtaChains c = chains_of(w);
  c.zn = E.zn;
  if (side) c.tail = TailWs{w.tws, kTailTiles, side->la.slots};  // the Schur updates on s
  SelinvChains si = selinv_of(w);
  si.zn = E.zn;
  // The gradient's side work runs block by block beside the sweep when the panels leave room
  // for it (side_beside_sweep), else after the sweep for all blocks at once (prepare_all):
  // beside panels that fill the CUs its long product tiles delay the next panel launch, and on
  // the look-ahead stream's hardware queue it delays the look-ahead updates behind it.
  const bool defer = w.defer && !side_beside_sweep(w, side);
  if (defer) c.invert = false;
  const bool fork = c.invert && side && w.slotsD >= 3;
  if (fork) {
    c.invert = false;
    c.inv_maxwg = side->side_maxwg;
    si.prep_maxwg = side->side_maxwg;
  }
  hipLaunchKernelGGL(assemble_blocks_kernel, agrid, dim3(64), 0, s, E.dev, 0, -1, w.D, w.zD,
                     w.Bin, w.zB, (long long)b, w.phi, w.tau);
  // B_i is assembled straight into the rows of [L_B; L_C] of block i instead of a separate
  // slot (then copied) when that slot is free before block i starts: a gradient keeps every
  // block's slot, an objective a ring of two
  const bool ring = !w.grad && w.slotsD >= 3 && w.slotsLBC >= 2;
  c.b_in_place = fork || defer || ring;
  const long long ldT = (long long)b + w.ap;
  // Fused steps (the look-ahead stream idle) and stored factors with the side work after the
  // sweep, or an objective's rings: D_{i+2} and B_{i+1} are assembled on the look-ahead stream
  // beside block i's last steps, which leave CUs idle (they only read theta, into slots no
  // launch of block i touches), so that block i+1 starts without them
  const int npanel = (b + kPanel - 1) / kPanel;
  const bool pre_asm = side && c.b_in_place &&
                       (defer ? w.slotsD == n && w.slotsLBC == n : ring) &&
                       1LL * nz * panel_workgroups(b, 0, b + w.ap) <= side->la.cus;
  for (int i = 0; i < n; ++i) {
    // the sweep stays at most two blocks ahead of the side stream (without this wait: 46.1
    // against 44.4 ms per gradient at b = 1024), which also keeps a ring of three D slots safe
    if (fork && i >= 2 && hipStreamWaitEvent(s, side->done[(i - 2) % 3], 0) != hipSuccess)
      return ADELIA_E_HIP;
    const int td = i + 1 < n ? i + 1 : -1;
    const int tb = i < n - 1 ? i : -1;
    if ((td >= 0 || tb >= 0) && pre_asm && i >= 1) {
      // assembled beside block i - 1
      if (hipStreamWaitEvent(s, side->la.tdone[i % 3], 0) != hipSuccess) return ADELIA_E_HIP;
    } else if (td >= 0 || tb >= 0) {
      double* Dslot = w.D + (long long)((i + 1) % w.slotsD) * w.sD;
      const bool inplace = c.b_in_place;
      double* Bslot = inplace ? w.LBC + (long long)(i % w.slotsLBC) * ldT * b : w.Bin;
      const ProfToken t = prof_begin(s);
      hipLaunchKernelGGL(assemble_blocks_kernel, agrid, dim3(64), 0, s, E.dev, td, tb, Dslot,
                         w.zD, Bslot, inplace ? w.zLBC : w.zB, inplace ? ldT : (long long)b,
                         w.phi, w.tau);
      if (t.valid) prof_end(t, s, PK_ASSEMBLE, 0.0, 8.0 * bb * nz * ((td >= 0) + (tb >= 0)));
      if (!LAUNCH_OK()) return ADELIA_E_HIP;
    }
    // The side work of block i-1 (its inversion and the selected-inversion preparation) is
    // forked after the first step of block i rather than right after block i-1: the first steps
    // of a block carry most of its update tiles and run faster without the side stream's
    // products beside them (measured 47.7 against 48.6 ms per gradient; forking after later
    // steps lets the side stream fall behind).
    Lookahead la{};
    if (side) la = side->la;
    la.mark = nullptr;
    const bool late = fork && i >= 1;
    if (late) {
      la.mark = side->ready[(i - 1) % 3];
      la.mark_step = 0;
    }
    const bool ahead = pre_asm && i + 2 < n;  // D_{i+2} and B_{i+1} exist
    if (ahead) {
      la.mark = side->la.pdone[i % 3];
      la.mark_step = std::max(0, npanel - 4);
    }
    // carry-only: the diagonal block about to be factored is D_i - S_{i-1}
    if (w.carry && launch_copy2d(w.D + (long long)(i % w.slotsD) * w.sD, b, w.zD,
                                 w.Dc + (long long)i * bb, b, w.zDc, b, b, nz, s))
      return ADELIA_E_HIP;
    if (bta_forward_block(c, i, s, side ? &la : nullptr)) return ADELIA_E_HIP;
    if (ahead) {
      hipStream_t ts = side->la.ts;
      if (hipStreamWaitEvent(ts, side->la.pdone[i % 3], 0) != hipSuccess) return ADELIA_E_HIP;
      const ProfToken t = prof_begin(ts);
      hipLaunchKernelGGL(assemble_blocks_kernel, agrid, dim3(64), 0, ts, E.dev, i + 2, i + 1,
                         w.D + (long long)((i + 2) % w.slotsD) * w.sD, w.zD,
                         w.LBC + (long long)((i + 1) % w.slotsLBC) * ldT * b, w.zLBC, ldT,
                         w.phi, w.tau);
      if (t.valid) prof_end(t, ts, PK_ASSEMBLE, 0.0, 16.0 * bb * nz);
      if (!LAUNCH_OK() || hipEventRecord(side->la.tdone[(i + 1) % 3], ts) != hipSuccess)
        return ADELIA_E_HIP;
    }
    if (w.carry && w.ap > 0 &&
        launch_copy2d(w.LBC + (long long)(i % w.slotsLBC) * ldT * b + b, ldT, w.zLBC,
                      w.LCz + (long long)i * w.ap * b, w.ap, w.zLCz, w.ap, b, nz, s))
      return ADELIA_E_HIP;
    auto fork_block = [&](int j, bool recorded) -> int {
      if ((!recorded && hipEventRecord(side->ready[j % 3], s) != hipSuccess) ||
          hipStreamWaitEvent(side->s2, side->ready[j % 3], 0) != hipSuccess)
        return ADELIA_E_HIP;
      if (bta_invert_block(c, j, side->s2)) return ADELIA_E_HIP;
      if (hipEventRecord(side->done[j % 3], side->s2) != hipSuccess) return ADELIA_E_HIP;
      if (prepare_block(E, w, si, j, side->s2)) return ADELIA_E_HIP;
      return 0;
    };
    if (fork) {
      if (late && fork_block(i - 1, true)) return ADELIA_E_HIP;
      if (i == n - 1 && fork_block(i, false)) return ADELIA_E_HIP;
    } else if (w.grad && !w.carry && !defer) {
      if (prepare_block(E, w, si, i, s)) return ADELIA_E_HIP;
    }
  }
  if (defer && prep && prepare_all(E, w, s)) return ADELIA_E_HIP;
  // the side stream runs its work in order: an event after its last product joins all of it
  if (fork && (hipEventRecord(side->done[n % 3], side->s2) != hipSuccess ||
               hipStreamWaitEvent(s, side->done[n % 3], 0) != hipSuccess))
    return ADELIA_E_HIP;
  if (tip && bta_tip(c, s)) return ADELIA_E_HIP;
  if (bta_logdet_reduce(w.ldpart, w.zLd, n * w.npanel + 1, w.ld, 1, nz, s)) return ADELIA_E_HIP;
  return 0;
}

// The upper sweep x = L^-T z over the factors kept in a gradient workspace (z_t is the rhs row
// of L_C).
SolveChains solve_of(const InlaWs& w) {
  const int n = w.n, b = w.b, a = w.a, ap = w.ap;
  SolveChains sc{};
  sc.n = n; sc.b = b; sc.a = a; sc.nz = w.nz;
  sc.G = w.G; sc.zG = w.zG; sc.slotsG = w.slotsG;
  const long long sLBC = (long long)(b + ap) * b;
  sc.LB = w.LBC; sc.zLB = w.zLBC; sc.slotsLB = w.slotsLBC; sc.ldLB = b + ap; sc.sLB = sLBC;
  sc.LC = w.LBC + b; sc.zLC = w.zLBC; sc.ldLC = b + ap; sc.sLC = sLBC;
  sc.z = w.LBC + b + a; sc.zz = w.zLBC; sc.sz_blk = sLBC; sc.sz_elem = b + ap;
  sc.xT = a ? w.xT : nullptr; sc.zxT = w.zXT;
  sc.x = w.x; sc.zx = w.zx;
  sc.y = w.y; sc.zy = w.zy;
  return sc;
}

int run_objective(const Eval& E, const InlaWs& w, const double* theta, double* f,
                  int32_t* info, hipStream_t s, const SideRes* side = nullptr) {
  int r = run_forward(E, w, theta, s, side);
  if (r) return r;
  hipLaunchKernelGGL(objective_kernel, dim3((w.batch + 63) / 64), dim3(64), 0, s, E.dev, theta,
                     w.batch, w.tau, w.ld, w.zsq, w.info, f, info);
  return LAUNCH_OK() ? 0 : ADELIA_E_HIP;
}

int run_backward(const Eval& E, const InlaWs& w, const double* theta, double* f, double* grad,
                 int32_t* info, double* terms, hipStream_t s, const SideRes* side) {
  const ModelDev& M = E.M;
  const int n = w.n, b = w.b, a = w.a, ap = w.ap, nz = w.nz;
  // x* = Qc^-1 r by the upper sweep (Eqs. 3-5); z_t is the rhs row of L_C
  SolveChains sc = solve_of(w);
  sc.zn = E.zn;
  // Only the mode of Qc (chain 2p of point p) is read (Phase B, the data residual): the upper
  // sweep runs on the Qc chains alone, seen as `batch` chains with doubled strides.
  auto qc_only = [&](SolveChains& c) {
    c.nz = w.batch;
    c.zG *= 2; c.zLB *= 2; c.zLC *= 2; c.zz *= 2; c.zxT *= 2; c.zx *= 2; c.zy *= 2;
    c.zn_stride = 2;
  };
  SelinvChains si = selinv_of(w);
  si.zn = E.zn;
  // selinv_finish's products run on one stream at a time (s, or s3 of the carry-only pass,
  // which starts after the forward sweep's Schur updates)
  if (side) si.tail = TailWs{w.tws, kTailTiles, side->la.slots};
  const long long bb = (long long)b * b;
  const int ntrace = 2 * M.k * M.k * M.nch_rows + M.k * M.nch_obs;
  auto trace = [&](int j, hipStream_t ts) -> int {
    const double* ZDj = w.ZD + (long long)(j % w.slotsZD) * bb;
    const double* ZCj = w.ZC + (long long)(j % 2) * a * b;
    const ProfToken t = prof_begin(ts);
    hipLaunchKernelGGL(trace_kernel, dim3(ntrace, 1, nz), dim3(256), 0, ts, E.dev, j, ZDj, w.zZD,
                       w.ZB, w.zZB, ZCj, w.zZC, w.ZT, w.zZT, w.TD, w.TB, w.O, w.zTr, w.zO);
    if (t.valid)  // the band of Z_D and Z_B at the base-matrix pattern, per sub-block pair
      prof_end(t, ts, PK_TRACE, 0.0, 8.0 * nz * 2.0 * M.k * M.k * M.nnz);
    return LAUNCH_OK() ? 0 : ADELIA_E_HIP;
  };
  bool forked = false;
  if (w.carry) {
    // Carry-only (Sec. III-A-2, L reconstruction): block j's factor is rebuilt from its stored
    // Schur-updated diagonal block D_j - S_{j-1} and B_j (assembled again from theta): the
    // panels solve B_j only (the arrow rows [L_C | z] are stored), then G_j, [W_j; V_j] and
    // G_j^T G_j, the upper-solve step for x_j and the selected-inversion step, all in one pass
    // from the last block down.
    sc.LC = w.LCz; sc.zLC = w.zLCz; sc.ldLC = ap; sc.sLC = (long long)ap * b;
    sc.z = w.LCz + a; sc.zz = w.zLCz; sc.sz_blk = (long long)ap * b; sc.sz_elem = ap;
    qc_only(sc);
    BtaChains c = chains_of(w);
    c.zn = E.zn;
    c.refactor = true;
    c.b_in_place = true;
    c.invert = false;
    Lookahead la{};
    if (side) {
      la = side->la;
      la.mark = nullptr;
    }
    const long long ldT = (long long)b + ap;
    const dim3 agrid(b, 1, nz);
    // Pipelined over three streams when the rebuild takes the single-launch steps (the
    // look-ahead stream is then free): rebuilding block j (main stream), its inverse and
    // [W_j; V_j], G_j^T G_j (side stream), and the upper-solve, selected-inversion and trace
    // steps (look-ahead stream) overlap for consecutive blocks.  The rebuild of block j reuses
    // the ring slots of block j+3, whose last reader is block j+2's selected-inversion step.
    const bool pipe = side && 2LL * nz * panel_workgroups(b, 0, b) <= side->la.cus;
    hipStream_t s2 = pipe ? side->s2 : s, s3 = pipe ? side->la.ts : s;
    // The selected-inversion stage runs beside the rebuild's latency-bound panel steps.  While
    // its Z_B product has at most two tiles per CU, its grids are capped at 3/8 of the CUs
    // (b = 1024: 88.4 -> 84.4 ms per gradient; caps of 72-104 workgroups measure alike, 112-128
    // less well).  Larger products set the pace themselves and stay uncapped (a cap of 144 at
    // b = 1200: 78.4 -> 81.0 ms; of 96 at b = 2700: 671 -> 996 ms).
    if (pipe) {
      const long long tiles = (long long)nz * ((b + 63) / 64) * ((b + 63) / 64);
      if (tiles <= 2LL * side->la.cus) si.fin_maxwg = std::max(8, (3 * side->la.cus / 8) & ~7);
    }
    const hipEvent_t* built = pipe ? side->ready : nullptr;
    const hipEvent_t* prepared = pipe ? side->la.pdone : nullptr;
    const hipEvent_t* finished = pipe ? side->la.tdone : nullptr;
    if (pipe && (hipEventRecord(side->done[0], s) != hipSuccess ||
                 hipStreamWaitEvent(s2, side->done[0], 0) != hipSuccess ||
                 hipStreamWaitEvent(s3, side->done[0], 0) != hipSuccess))
      return ADELIA_E_HIP;
    for (int j = n - 1; j >= 0; --j) {
      if (pipe && j + 2 <= n - 1 && hipStreamWaitEvent(s, finished[(j + 2) % 3], 0) != hipSuccess)
        return ADELIA_E_HIP;
      double* Dslot = w.D + (long long)(j % w.slotsD) * w.sD;
      if (launch_copy2d(w.Dc + (long long)j * bb, b, w.zDc, Dslot, b, w.zD, b, b, nz, s))
        return ADELIA_E_HIP;
      if (j < n - 1) {
        hipLaunchKernelGGL(assemble_blocks_kernel, agrid, dim3(64), 0, s, E.dev, -1, j, Dslot, w.zD,
                           w.LBC + (long long)(j % w.slotsLBC) * ldT * b, w.zLBC, ldT, w.phi,
                           w.tau);
        if (!LAUNCH_OK()) return ADELIA_E_HIP;
      }
      if (bta_forward_block(c, j, s, side ? &la : nullptr)) return ADELIA_E_HIP;
      if (pipe && (hipEventRecord(built[j % 3], s) != hipSuccess ||
                   hipStreamWaitEvent(s2, built[j % 3], 0) != hipSuccess))
        return ADELIA_E_HIP;
      if (bta_invert_block(c, j, s2) || prepare_block(E, w, si, j, s2)) return ADELIA_E_HIP;
      if (pipe && (hipEventRecord(prepared[j % 3], s2) != hipSuccess ||
                   hipStreamWaitEvent(s3, prepared[j % 3], 0) != hipSuccess))
        return ADELIA_E_HIP;
      if (bta_upper_solve_block(sc, j, s3) || selinv_finish(si, j, s3)) return ADELIA_E_HIP;
      if (int r = trace(j, s3)) return r;
      if (pipe && hipEventRecord(finished[j % 3], s3) != hipSuccess) return ADELIA_E_HIP;
    }
    if (pipe && hipStreamWaitEvent(s, finished[0], 0) != hipSuccess) return ADELIA_E_HIP;
    if (bta_upper_solve_tip(sc, s)) return ADELIA_E_HIP;
  } else {
    qc_only(sc);
    // x* is read only by Phase B and the residual at the end: with the side stream (idle after
    // the forward sweep's join) the upper sweep runs there, beside the selected inversion
    if (side) {
      if (hipEventRecord(side->ready[0], s) != hipSuccess ||
          hipStreamWaitEvent(side->s2, side->ready[0], 0) != hipSuccess ||
          bta_upper_solve(sc, side->s2) ||
          hipEventRecord(side->done[0], side->s2) != hipSuccess)
        return ADELIA_E_HIP;
      forked = true;
    } else if (bta_upper_solve(sc, s)) {
      return ADELIA_E_HIP;
    }
    // selected inversion of Qc and Qp with the trace epilogue per block (Eq. 6); the forward
    // sweep already formed [W_j; V_j] and G_j^T G_j
    for (int j = n - 1; j >= 0; --j) {
      if (selinv_finish(si, j, s)) return ADELIA_E_HIP;
      if (int r = trace(j, s)) return r;
    }
  }
  if (forked && hipStreamWaitEvent(s, side->done[0], 0) != hipSuccess) return ADELIA_E_HIP;
  // Phase B (Eq. 8) and the likelihood residual, from the mode of Qc (chain 2p of point p)
  const int B = w.batch;
  hipLaunchKernelGGL(phaseb_kernel, dim3(n * M.k, 1, B), dim3(256), 0, s, E.dev, w.x, 2 * w.zx,
                     w.qD, w.qB, w.zq);
  hipLaunchKernelGGL(resid_kernel, dim3(M.k * M.nch_resid, 1, B), dim3(256), 0, s, E.dev, w.x,
                     2 * w.zx, w.n, w.resid, w.zr);
  hipLaunchKernelGGL(grad_kernel, dim3(B), dim3(256), 0, s, E.dev, theta, w.dphi, w.tau, w.TD, w.TB,
                     w.zTr, w.O, w.zO, w.qD, w.qB, w.zq, w.resid, w.zr, w.ld, w.zsq, w.ZT, w.zZT,
                     w.info, f, grad, info, B == 1 ? terms : nullptr);
  return LAUNCH_OK() ? 0 : ADELIA_E_HIP;
}

bool aligned(const void* p, size_t al) { return ((uintptr_t)p % al) == 0; }

// Kernel launches of one batched pass (objective, or gradient with its reverse pass) over
// `batch` points, from the schedule rules of the sweeps: per block the assembly and arrow copy,
// the panel launches (fused steps: one per panel; split panels: the diagonal tile, its rows'
// GEMM and the trailing update; otherwise panel plus trailing update), the Schur update, and for
// a gradient the inversion (two GEMMs per doubling level), the selected-inversion preparation
// (three), its finish with the trace (four) and the upper solve (two).  Counted per block, an
// upper bound: a stored-factor gradient runs the inversion and the preparation once for all
// blocks.
long long launches_per_pass(const ModelDev& M, const SideRes* side, int batch, bool grad) {
  const int b = M.b, ap = M.a + 1, nz = 2 * batch;
  const int npanel = (b + kPanel - 1) / kPanel;
  const int cus = side ? side->la.cus : 256;
  const long long wg = (long long)nz * panel_workgroups(b, 0, b + ap);
  const int per_panel = side && wg <= cus ? 1 : (wg > cus ? 3 : 2);
  int levels = 0;
  for (int sz = kPanel; sz < b; sz *= 2) ++levels;
  long long per_block = 4 + (long long)per_panel * npanel;
  if (grad) per_block += 2 * levels + 3 + 6 + 2;
  return 16 + (long long)M.nt * per_block;
}

// Capturing very long calls into one graph: an FD Hessian at b = 2700, d = 15 (15 passes of 31
// points, about 96,000 launches by the estimate above) ended the process with a host
// segmentation fault during the capture or its first replay, while captures of up to about
// 44,000 estimated launches (the Eq. 12 Hessian at the same size) run normally.  The cause has
// not been established (no GPU fault was reported; the same calls run eagerly).  Until it is,
// a call whose estimated launch count exceeds this bound returns ADELIA_E_UNSUPPORTED when
// its stream is capturing, before anything is enqueued.
constexpr long long kCaptureLaunchLimit = 60000;

int capture_guard(hipStream_t s, long long planned) {
  if (planned <= kCaptureLaunchLimit) return 0;
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) {
    (void)hipGetLastError();  // a failed query must not read as a failed launch later
    return 0;
  }
  return st == hipStreamCaptureStatusNone ? 0 : ADELIA_E_UNSUPPORTED;
}

int fail(const std::string& msg) {
  set_last_error(msg);
  return ADELIA_E_SHAPE;
}

// CSR validation; returns an empty string when valid
std::string check_csr(const char* name, const int32_t* ptr, const int32_t* idx, const double* val,
                      int ns) {
  if (!ptr || !idx || !val) return std::string(name) + ": null CSR array";
  if (ptr[0] != 0) return std::string(name) + ": row pointer must start at 0";
  for (int r = 0; r < ns; ++r) {
    if (ptr[r + 1] < ptr[r]) return std::string(name) + ": row pointer decreases";
    for (int e = ptr[r]; e < ptr[r + 1]; ++e)
      if (idx[e] < 0 || idx[e] >= ns) return std::string(name) + ": column index out of range";
  }
  // symmetry (values included)
  std::map<std::pair<int, int>, double> ent;
  for (int r = 0; r < ns; ++r)
    for (int e = ptr[r]; e < ptr[r + 1]; ++e) ent[{r, idx[e]}] += val[e];
  for (const auto& kv : ent) {
    auto it = ent.find({kv.first.second, kv.first.first});
    if (it == ent.end() || it->second != kv.second) return std::string(name) + ": not symmetric";
  }
  return "";
}

}  // namespace

namespace {

// ---- uneven batches of INLA instances -------------------------------------------------------
// Instances with the same block size b (and k, parameterisation, d) form a group whose chains
// share every launch.  Inside a group the arrow is padded to the largest a with zero covariate
// columns (the padded fixed effects keep their prior precision in Qp and Qc alike, are decoupled
// from everything else and have no theta dependence, so f and its gradient are unchanged:
// their log-determinant terms cancel between Qp and Qc and every other term is zero), and an
// instance with fewer blocks drops out of the sweeps past its last block (per-chain block
// counts; its coupling block after the last one is zero).  Groups run one after another.
struct BatchGroup {
  ModelDev Mh;  // sizes of the group's layout: the largest nt, a, observation slices
  ModelDev* Mv = nullptr;     // device: one model per member (a padded to the group's)
  int32_t* zn = nullptr;      // device: block count per chain (2 per member)
  int32_t* idx = nullptr;     // device: the member's position in the batch
  std::vector<int> members;
};

__global__ void gather_rows_kernel(const double* src, int d, const int32_t* idx, int n,
                                   double* dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * d) return;
  dst[i] = src[(long long)idx[i / d] * d + i % d];
}

__global__ void scatter_results_kernel(const double* f, const double* g, const int32_t* info,
                                       int n, int d, const int32_t* idx, double* f_out,
                                       double* g_out, int32_t* info_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * d) return;
  const int p = i / d, c = i % d, q = idx[p];
  if (g_out) g_out[(long long)q * d + c] = g[i];
  if (c == 0) {
    f_out[q] = f[p];
    info_out[q] = info[p];
  }
}

// X (n_obs x a, row-major) copied into n_obs x ap columns, the extra columns zero
__global__ void pad_cols_kernel(const double* X, int n_obs, int a, int ap, double* Xp) {
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= (long long)n_obs * ap) return;
  const long long o = i / ap;
  const int c = (int)(i % ap);
  Xp[i] = c < a ? X[o * a + c] : 0.0;
}

// Zero block slot zn[z] of every chain z with zn[z] < nmax (the Z_D block after an instance's
// last block, read with a zero factor when its last block is inverted).
__global__ void zero_next_slot_kernel(double* Z, long long zZ, long long slot, const int32_t* zn,
                                      int nmax) {
  const int z = blockIdx.z;
  const int nzb = zn[z];
  if (nzb >= nmax) return;
  double* p = Z + (long long)z * zZ + (long long)nzb * slot;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < slot; e += (long long)gridDim.x * 256)
    p[e] = 0.0;
}

// Scratch in front of a batch workspace: the gathered points and the group's results.
struct BatchFront {
  double *Th, *fv, *gv;
  int32_t* finfo;
  size_t bytes;
};

BatchFront batch_front(int count, int d, char* base) {
  BatchFront b{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off = align_up(off + bytes);
    return p;
  };
  b.Th = reinterpret_cast<double*>(take((size_t)count * d * 8));
  b.fv = reinterpret_cast<double*>(take((size_t)count * 8));
  b.gv = reinterpret_cast<double*>(take((size_t)count * d * 8));
  b.finfo = reinterpret_cast<int32_t*>(take((size_t)count * 4));
  b.bytes = off;
  return b;
}

}  // namespace

struct inla_batch_s {
  int device, d, count;
  std::vector<BatchGroup> groups;
  void* dev_mem;
  SideRes side;
  bool has_side;
};

namespace {

size_t batch_ws_bytes(const inla_batch_s* B, bool grad) {
  size_t most = 0;
  for (const BatchGroup& g : B->groups)
    most = std::max(most, layout(g.Mh, (int)g.members.size(), grad, nullptr).bytes);
  return batch_front(B->count, B->d, nullptr).bytes + most;
}

// Groups [g0, g1) of the batch (all: g1 < 0).  f == nullptr: results stay in the workspace
// (timing runs of the autotuner); with_grad selects gradients.
int batch_eval(inla_batch_s* B, const double* theta, double* f, double* grad, int32_t* info,
               void* ws, hipStream_t s, bool with_grad, int g0 = 0, int g1 = -1) {
  char* base = reinterpret_cast<char*>(ws);
  const BatchFront fr = batch_front(B->count, B->d, base);
  const SideRes* side = B->has_side ? &B->side : nullptr;
  const int d = B->d;
  if (g1 < 0) g1 = (int)B->groups.size();
  for (int gi = g0; gi < g1; ++gi) {
    const BatchGroup& g = B->groups[gi];
    const int ng = (int)g.members.size();
    InlaWs w = layout(g.Mh, ng, with_grad, base + fr.bytes);
    hipLaunchKernelGGL(gather_rows_kernel, dim3((ng * d + 255) / 256), dim3(256), 0, s, theta, d,
                       g.idx, ng, fr.Th);
    if (!LAUNCH_OK()) return ADELIA_E_HIP;
    // what the skipped steps of shorter instances would have written: zero log-determinant
    // partials, and for the reverse pass a zero x and Z_C and a zero Z_D block after each
    // instance's last block
    if (launch_fill(w.ldpart, (long long)w.nz * w.zLd, 0.0, s)) return ADELIA_E_HIP;
    const Eval E{g.Mh, Models{g.Mv, 1}, g.zn};
    int r;
    if (!with_grad) {
      r = run_objective(E, w, fr.Th, fr.fv, fr.finfo, s, side);
    } else {
      const long long bb = (long long)w.b * w.b;
      if (launch_fill(w.x, (long long)w.nz * w.zx, 0.0, s) ||
          launch_fill(w.ZC, (long long)w.nz * w.zZC, 0.0, s))
        return ADELIA_E_HIP;
      hipLaunchKernelGGL(zero_next_slot_kernel, dim3(std::max(1, (int)std::min<long long>(bb / 256, 256)), 1, w.nz),
                         dim3(256), 0, s, w.ZD, w.zZD, bb, g.zn, w.n);
      if (!LAUNCH_OK()) return ADELIA_E_HIP;
      r = run_forward(E, w, fr.Th, s, side);
      if (!r) r = run_backward(E, w, fr.Th, fr.fv, fr.gv, fr.finfo, nullptr, s, side);
    }
    if (r) return r;
    if (!f) continue;
    hipLaunchKernelGGL(scatter_results_kernel, dim3((ng * d + 255) / 256), dim3(256), 0, s, fr.fv,
                       fr.gv, fr.finfo, ng, d, g.idx, f, grad, info);
    if (!LAUNCH_OK()) return ADELIA_E_HIP;
  }
  return 0;
}

// The roles whose tile edge the autotuners choose (the update part of a fused look-ahead step
// always takes 64 x 64 tiles).
// The panel-rows product of the split schedule, formed in place, keeps 64 x 64 tiles.
constexpr int kTunedRoles[] = {GT_TRAIL, GT_TRTRI, GT_SYRK, GT_SI_W, GT_SI_Z, GT_SI_D};

// Coordinate search over the roles at block size b: each role in turn tries 64 and 32 with the
// other roles as chosen so far, timing `reps` runs of eval() (after one untimed run) with events
// on s; a role switches only for a gain of more than 2%.  Returns 0 or ADELIA_E_HIP; *changed
// counts the roles whose choice differs from before.
template <class F>
int tune_block_size(int b, F&& eval, int reps, hipStream_t s, int* changed) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return ADELIA_E_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return ADELIA_E_HIP;
  }
  auto run_ms = [&](float& ms) -> int {
    if (eval()) return ADELIA_E_HIP;
    std::vector<float> t;
    for (int r = 0; r < reps; ++r) {
      if (hipEventRecord(e0, s) != hipSuccess || eval() || hipEventRecord(e1, s) != hipSuccess ||
          hipEventSynchronize(e1) != hipSuccess)
        return ADELIA_E_HIP;
      float v = 0.f;
      if (hipEventElapsedTime(&v, e0, e1) != hipSuccess) return ADELIA_E_HIP;
      t.push_back(v);
    }
    std::sort(t.begin(), t.end());
    ms = t[t.size() / 2];
    return 0;
  };
  int err = 0;
  for (int role : kTunedRoles) {
    const int before = tuned_tile(b, role);
    int best = before;
    float best_ms = 0.f;
    if ((err = run_ms(best_ms))) break;
    for (int tile : {64, 32}) {
      if (tile == before) continue;
      set_tuned_tile(b, role, tile);
      float ms = 0.f;
      if ((err = run_ms(ms))) break;
      if (ms < 0.98f * best_ms) {
        best = tile;
        best_ms = ms;
      }
    }
    set_tuned_tile(b, role, best);
    if (err) break;
    if (best != before) ++*changed;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return err;
}

long long batch_launches(const inla_batch_s* B, bool grad) {
  long long t = 0;
  for (const BatchGroup& g : B->groups)
    t += 8 + launches_per_pass(g.Mh, B->has_side ? &B->side : nullptr, (int)g.members.size(), grad);
  return t;
}

}  // namespace


// The side stream, the look-ahead stream and their events (default priority), for the device
// `device` (current).  The side stream's products (inversion, selected-inversion preparation)
// run beside the panels of the sweep, whose workgroups each need a CU of their own (most of its
// LDS): they are capped at 5/8 of the CUs in tile slots, two tiles per workgroup
// (gemm_f64_dual_kernel), i.e. on 5/16 of the CUs (measured on 256 CUs: 144-168 slots all best,
// 128 and 176 clearly worse).
static bool make_side(SideRes& sr, int device) {
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
      cus <= 0)
    cus = 256;
  sr.la.maxwg = 0;
  sr.la.cus = cus;
  sr.la.slots = cus * gemm_resident_per_cu();
  sr.la.mark = nullptr;
  sr.la.mark_step = 0;
  sr.side_maxwg = std::max(16, (5 * cus / 8) & ~15);
  bool ok = hipStreamCreateWithFlags(&sr.s2, hipStreamNonBlocking) == hipSuccess &&
            hipStreamCreateWithFlags(&sr.la.ts, hipStreamNonBlocking) == hipSuccess;
  for (int e = 0; e < 3 && ok; ++e)
    ok = hipEventCreateWithFlags(&sr.ready[e], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&sr.done[e], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&sr.la.pdone[e], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&sr.la.tdone[e], hipEventDisableTiming) == hipSuccess;
  return ok;
}

static void free_side(SideRes& sr) {
  hipStreamSynchronize(sr.s2);
  hipStreamSynchronize(sr.la.ts);
  for (int e = 0; e < 3; ++e) {
    hipEventDestroy(sr.ready[e]);
    hipEventDestroy(sr.done[e]);
    hipEventDestroy(sr.la.pdone[e]);
    hipEventDestroy(sr.la.tdone[e]);
  }
  hipStreamDestroy(sr.s2);
  hipStreamDestroy(sr.la.ts);
}

static Eval eval_of(inla_model m) { return Eval{m->M, Models{m->Md, 0}, nullptr}; }

// ---- two-sided split (one gradient or objective) ----------------------------------------------
// Workspace: theta twice (one row per half), the halves' results, the halves' layout (two
// points: chains A-Qc, A-Qp, B-Qc, B-Qp) and the reduced system's (one block, chains Qc, Qp).
struct SplitWs {
  double *Th2, *fv, *gv;
  int32_t* finfo;
  InlaWs h, r;
  size_t bytes;
};

static SplitWs split_layout(const inla_model_s* m, bool grad, char* base) {
  SplitWs w{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off = align_up(off + bytes);
    return p;
  };
  const int d = m->M.d;
  w.Th2 = reinterpret_cast<double*>(take((size_t)2 * d * 8));
  w.fv = reinterpret_cast<double*>(take(2 * 8));
  w.gv = reinterpret_cast<double*>(take((size_t)2 * d * 8));
  w.finfo = reinterpret_cast<int32_t*>(take(2 * 4));
  w.h = layout(m->Mh, 2, grad, base ? base + off : nullptr);
  off = align_up(off + w.h.bytes);
  w.r = layout(m->Mr, 1, grad, base ? base + off : nullptr);
  off = align_up(off + w.r.bytes);
  w.bytes = off;
  return w;
}

// One objective (grad == nullptr) or gradient by the two-sided split: both halves' sweeps in the
// same launches, toward the separator (Phase 1 of Sec. III-C); the separator block, its arrow
// rows and the tip summed over the halves and factored as the reduced system (Phase 2); for the
// gradient, the reduced system's selected inverse and mode seed both halves' reverse passes,
// whose gradients add up.
static int run_split(inla_model m, const SplitWs& sw, const double* theta, double* f,
                     double* grad, int32_t* info, hipStream_t s) {
  const SideRes* side = m->has_side ? &m->side : nullptr;
  const Eval Eh{m->Mh, Models{m->half_dev, 1}, m->zn_split};
  const InlaWs& h = sw.h;
  const InlaWs& r = sw.r;
  const int d = m->M.d, b = h.b, a = h.a, ap = h.ap;
  const bool with_grad = grad != nullptr;
  for (int q = 0; q < 2; ++q)
    if (launch_copy2d(theta, d, 0, sw.Th2 + q * d, d, 0, d, 1, 1, s)) return ADELIA_E_HIP;
  // the separator's panels and the halves' tips are never factored: zero partials
  if (launch_fill(h.ldpart, (long long)h.nz * h.zLd, 0.0, s)) return ADELIA_E_HIP;
  if (with_grad && (launch_fill(h.x, (long long)h.nz * h.zx, 0.0, s) ||
                    launch_fill(h.ZC, (long long)h.nz * h.zZC, 0.0, s)))
    return ADELIA_E_HIP;
  if (int e = run_forward(Eh, h, sw.Th2, s, side, false, false)) return e;
  // the halves' selected-inversion preparation (every block but the separator, which belongs
  // to the reduced system) runs on the side stream beside the reduced system's factorisation,
  // whose two chains leave most CUs idle
  const bool deferred = with_grad && !side_beside_sweep(h, side);
  const bool fork_prep = deferred && side;
  if (fork_prep && (hipEventRecord(side->ready[1], s) != hipSuccess ||
                    hipStreamWaitEvent(side->s2, side->ready[1], 0) != hipSuccess ||
                    prepare_all(Eh, h, side->s2) ||
                    hipEventRecord(side->done[1], side->s2) != hipSuccess))
    return ADELIA_E_HIP;
  if (deferred && !side && prepare_all(Eh, h, s)) return ADELIA_E_HIP;
  const long long bb = (long long)b * b;
  const long long tot = bb + (long long)ap * b + (long long)ap * ap;
  hipLaunchKernelGGL(split_merge_kernel, dim3((unsigned)std::min<long long>((tot + 255) / 256, 1024), 1, 2),
                     dim3(256), 0, s, h.D, h.zD, h.sD, h.slotsD, h.C, h.zC, (long long)ap * b, h.T,
                     h.zT, m->zn_split, b, ap, r.D, r.zD, r.C, r.zC, r.T, r.zT);
  if (!LAUNCH_OK()) return ADELIA_E_HIP;
  // the reduced system: one block with the arrow and the tip
  BtaChains cr = chains_of(r);
  cr.b_in_place = false;
  if (launch_fill_i32(r.info, r.nz, INT32_MAX, s) || launch_fill_i32(r.cnt, r.nz, 0, s))
    return ADELIA_E_HIP;
  Lookahead la{};
  if (side) {
    la = side->la;
    la.mark = nullptr;
  }
  if (bta_forward_block(cr, 0, s, side ? &la : nullptr) || bta_tip(cr, s) ||
      bta_logdet_reduce(r.ldpart, r.zLd, r.npanel + 1, r.ld, 1, r.nz, s))
    return ADELIA_E_HIP;
  if (!with_grad) {
    hipLaunchKernelGGL(split_combine_kernel, dim3(1), dim3(64), 0, s, Models{m->Md, 0}, theta,
                       h.tau, h.ld, r.ld, r.zsq, h.info, r.info, nullptr, nullptr, f, nullptr,
                       info);
    return LAUNCH_OK() ? 0 : ADELIA_E_HIP;
  }
  // the reduced system's selected inverse and its part of the mode
  const SelinvChains sir = selinv_of(r);
  if (selinv_prepare(sir, 0, s) || selinv_finish(sir, 0, s)) return ADELIA_E_HIP;
  SolveChains scr = solve_of(r);
  scr.nz = 1;  // the mode of Qc only
  if (bta_upper_solve(scr, s)) return ADELIA_E_HIP;
  const long long stot = bb + (long long)a * b + (long long)a * a + b + a;
  hipLaunchKernelGGL(split_seed_kernel, dim3((unsigned)std::min<long long>((stot + 255) / 256, 1024), 1, h.nz),
                     dim3(256), 0, s, r.ZD, r.zZD, r.ZC, r.zZC, r.ZT, r.zZT, r.x, r.zx, r.xT,
                     r.zXT, b, a, m->zn_split, h.slotsZD, h.ZD, h.zZD, h.ZC, h.zZC, h.ZT, h.zZT,
                     h.x, h.zx, h.xT, h.zXT);
  if (!LAUNCH_OK()) return ADELIA_E_HIP;
  if (fork_prep && hipStreamWaitEvent(s, side->done[1], 0) != hipSuccess) return ADELIA_E_HIP;
  if (int e = run_backward(Eh, h, sw.Th2, sw.fv, sw.gv, sw.finfo, nullptr, s, side)) return e;
  hipLaunchKernelGGL(split_combine_kernel, dim3(1), dim3(64), 0, s, Models{m->Md, 0}, theta,
                     h.tau, h.ld, r.ld, r.zsq, h.info, r.info, sw.gv, sw.finfo, f, grad, info);
  return LAUNCH_OK() ? 0 : ADELIA_E_HIP;
}

// Estimated launches of `npts` points evaluated in passes of at most `bmax` points.
static long long planned_passes(inla_model m, int npts, int bmax, bool grad) {
  const SideRes* side = m->has_side ? &m->side : nullptr;
  const long long full = npts / bmax, rest = npts % bmax;
  return full * launches_per_pass(m->M, side, bmax, grad) +
         (rest ? launches_per_pass(m->M, side, (int)rest, grad) : 0);
}

extern "C" {

static int build_split(adelia_ctx ctx, const inla_model_desc* d, inla_model m);

static int model_create_impl(adelia_ctx ctx, const inla_model_desc* d, inla_model* out,
                             bool full) {
  if (!ctx) return -1;
  if (!d) return -2;
  if (!out) return -3;
  if (d->param != ADELIA_PARAM_UNIVARIATE && d->param != ADELIA_PARAM_COREG)
    return fail("unknown parameterisation");
  const int k = d->k, ns = d->ns, nt = d->nt, a = d->a, n_obs = d->n_obs;
  if (k < 1 || k > kMaxFields) return fail("k must be 1..4");
  if (d->param == ADELIA_PARAM_UNIVARIATE && k != 1) return fail("univariate model needs k == 1");
  if (ns < 1 || nt < 1 || a < 0 || a > 64 || n_obs < 0) return fail("bad sizes");
  const long long b = (long long)k * ns;
  if (b * nt + a > INT_MAX) return fail("model too large");
  if (b > kMaxBlock) return fail("block size k*ns above 16320 (a GEMM operand would pass 2 GiB)");
  if (!(d->sigma_prior > 0.0) || !(d->tip_prec > 0.0)) return fail("sigma and tip_prec must be > 0");
  std::string e;
  if (!(e = check_csr("c0", d->c0_ptr, d->c0_idx, d->c0_val, ns)).empty()) return fail(e);
  if (!(e = check_csr("g1", d->g1_ptr, d->g1_idx, d->g1_val, ns)).empty()) return fail(e);
  if (!(e = check_csr("g2", d->g2_ptr, d->g2_idx, d->g2_val, ns)).empty()) return fail(e);
  if (!d->m0_diag || !d->m1_diag || !d->m2_diag) return fail("null temporal diagonal");
  if (nt > 1 && (!d->m0_off || !d->m1_off || !d->m2_off)) return fail("null temporal sub-diagonal");
  if (n_obs > 0 && (!d->obs_t || !d->obs_field || !d->obs_node || !d->obs_w || !d->y))
    return fail("null observation array");
  if (n_obs > 0 && a > 0 && !d->X) return fail("null covariate matrix");
  long long prev = -1;
  for (int o = 0; o < n_obs; ++o) {
    const int t = d->obs_t[o], m = d->obs_field[o];
    if (t < 0 || t >= nt || m < 0 || m >= k) return fail("observation time/field out of range");
    const long long key = (long long)t * k + m;
    if (key < prev) return fail("observations must be sorted by (time, field)");
    prev = key;
    for (int q = 0; q < 4; ++q)
      if (d->obs_node[4 * o + q] < 0 || d->obs_node[4 * o + q] >= ns)
        return fail("observation node out of range");
  }
  // union pattern of the three base matrices
  std::vector<int32_t> uptr(ns + 1, 0), uidx;
  std::vector<double> u0, u1, u2;
  const int32_t* ptrs[3] = {d->c0_ptr, d->g1_ptr, d->g2_ptr};
  const int32_t* idxs[3] = {d->c0_idx, d->g1_idx, d->g2_idx};
  const double* vals[3] = {d->c0_val, d->g1_val, d->g2_val};
  for (int r = 0; r < ns; ++r) {
    std::map<int, double> row[3];
    std::vector<int> cols;
    for (int s = 0; s < 3; ++s)
      for (int q = ptrs[s][r]; q < ptrs[s][r + 1]; ++q) {
        row[s][idxs[s][q]] += vals[s][q];
        cols.push_back(idxs[s][q]);
      }
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    for (int c : cols) {
      uidx.push_back(c);
      u0.push_back(row[0].count(c) ? row[0][c] : 0.0);
      u1.push_back(row[1].count(c) ? row[1][c] : 0.0);
      u2.push_back(row[2].count(c) ? row[2][c] : 0.0);
    }
    uptr[r + 1] = (int32_t)uidx.size();
  }
  const int nnz = (int)uidx.size();
  // per tile of kWRows pattern rows: the pattern columns [lo, hi) its rows touch
  const int wtiles = (ns + kWRows - 1) / kWRows;
  std::vector<int32_t> wband(2 * (size_t)wtiles, 0);
  int wband_w = 1, wdeg = 0;
  for (int tt = 0; tt < wtiles; ++tt) {
    int lo = INT_MAX, hi = INT_MIN;
    for (int r = tt * kWRows; r < std::min(ns, (tt + 1) * kWRows); ++r) {
      wdeg = std::max(wdeg, uptr[r + 1] - uptr[r]);
      for (int e = uptr[r]; e < uptr[r + 1]; ++e) {
        lo = std::min(lo, uidx[e]);
        hi = std::max(hi, uidx[e] + 1);
      }
    }
    if (lo > hi) lo = 0, hi = 1;  // no entries
    wband[2 * tt] = lo;
    wband[2 * tt + 1] = hi;
    wband_w = std::max(wband_w, hi - lo);
  }
  std::vector<double> uval;
  uval.insert(uval.end(), u0.begin(), u0.end());
  uval.insert(uval.end(), u1.begin(), u1.end());
  uval.insert(uval.end(), u2.begin(), u2.end());
  std::vector<double> tm(3 * (2 * nt - 1), 0.0);
  const double* diags[3] = {d->m0_diag, d->m1_diag, d->m2_diag};
  const double* offs[3] = {d->m0_off, d->m1_off, d->m2_off};
  for (int r = 0; r < 3; ++r) {
    for (int t = 0; t < nt; ++t) tm[r * (2 * nt - 1) + t] = diags[r][t];
    for (int t = 0; t < nt - 1; ++t) tm[r * (2 * nt - 1) + nt + t] = offs[r][t];
  }
  std::vector<int32_t> obs_off(nt * k + 1, 0);
  std::vector<int32_t> nobs(k, 0);
  for (int o = 0; o < n_obs; ++o) {
    obs_off[d->obs_t[o] * k + d->obs_field[o] + 1]++;
    nobs[d->obs_field[o]]++;
  }
  for (int i = 0; i < nt * k; ++i) obs_off[i + 1] += obs_off[i];
  const long long ncolg = (long long)nt * b;
  std::vector<int32_t> colptr(ncolg + 1, 0);
  for (int o = 0; o < n_obs; ++o)
    for (int q = 0; q < 4; ++q) {
      const long long g = (long long)d->obs_t[o] * b + (long long)d->obs_field[o] * ns + d->obs_node[4 * o + q];
      colptr[g + 1]++;
    }
  for (long long g = 0; g < ncolg; ++g) colptr[g + 1] += colptr[g];
  std::vector<int32_t> col_o(colptr[ncolg]), col_e(colptr[ncolg]);
  {
    std::vector<int32_t> fillp(colptr.begin(), colptr.end() - 1);
    for (int o = 0; o < n_obs; ++o)
      for (int q = 0; q < 4; ++q) {
        const long long g = (long long)d->obs_t[o] * b + (long long)d->obs_field[o] * ns + d->obs_node[4 * o + q];
        col_o[fillp[g]] = o;
        col_e[fillp[g]] = q;
        fillp[g]++;
      }
  }
  // device upload: one allocation, set-up time only
  std::vector<std::pair<const void*, size_t>> parts = {
      {uptr.data(), uptr.size() * 4},    {uidx.data(), uidx.size() * 4},
      {uval.data(), uval.size() * 8},    {tm.data(), tm.size() * 8},
      {d->obs_t, (size_t)n_obs * 4},     {d->obs_field, (size_t)n_obs * 4},
      {d->obs_node, (size_t)n_obs * 16}, {d->obs_w, (size_t)n_obs * 32},
      {d->X, (size_t)n_obs * a * 8},     {d->y, (size_t)n_obs * 8},
      {obs_off.data(), obs_off.size() * 4}, {colptr.data(), colptr.size() * 4},
      {col_o.data(), col_o.size() * 4},  {col_e.data(), col_e.size() * 4},
      {nullptr, (size_t)k * 8},          {nullptr, sizeof(ModelDev)},
      {wband.data(), wband.size() * 4}};
  size_t total = 0;
  std::vector<size_t> offsets;
  for (auto& pr : parts) {
    offsets.push_back(total);
    total = align_up(total + std::max<size_t>(pr.second, 8));
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return ADELIA_E_HIP;
  char* mem = nullptr;
  if (hipMalloc(&mem, total) != hipSuccess) return ADELIA_E_HIP;
  for (size_t i = 0; i < parts.size(); ++i)
    if (parts[i].first && parts[i].second &&
        hipMemcpy(mem + offsets[i], parts[i].first, parts[i].second, hipMemcpyHostToDevice) != hipSuccess) {
      hipFree(mem);
      return ADELIA_E_HIP;
    }
  inla_model m = new inla_model_s();  // value-initialised: every handle starts null
  m->device = ctx->device;
  m->param = d->param;
  m->dev_mem = mem;
  ModelDev& M = m->M;
  std::memset(&M, 0, sizeof(M));
  M.k = k; M.ns = ns; M.nt = nt; M.a = a; M.b = (int)b; M.n_obs = n_obs; M.nnz = nnz;
  M.nch_rows = (ns + kTraceRows - 1) / kTraceRows;
  M.nch_resid = std::max(1, (n_obs + kResidObs - 1) / kResidObs);
  {
    int most = 0;
    for (int i = 0; i < nt * k; ++i) most = std::max(most, obs_off[i + 1] - obs_off[i]);
    M.nch_obs = std::max(1, (most + kTraceObs - 1) / kTraceObs);
  }
  M.sigma = d->sigma_prior; M.tip = d->tip_prec;
  M.uptr = (const int32_t*)(mem + offsets[0]);
  M.uidx = (const int32_t*)(mem + offsets[1]);
  M.uval = (const double*)(mem + offsets[2]);
  M.tm = (const double*)(mem + offsets[3]);
  M.obs_t = (const int32_t*)(mem + offsets[4]);
  M.obs_f = (const int32_t*)(mem + offsets[5]);
  M.obs_node = (const int32_t*)(mem + offsets[6]);
  M.obs_w = (const double*)(mem + offsets[7]);
  M.X = (const double*)(mem + offsets[8]);
  M.y = (const double*)(mem + offsets[9]);
  M.obs_off = (const int32_t*)(mem + offsets[10]);
  M.colptr = (const int32_t*)(mem + offsets[11]);
  M.col_o = (const int32_t*)(mem + offsets[12]);
  M.col_e = (const int32_t*)(mem + offsets[13]);
  M.yy = (const double*)(mem + offsets[14]);
  M.wband = (const int32_t*)(mem + offsets[16]);
  M.wband_w = wband_w;
  M.wdeg = wdeg;
  for (int i = 0; i < k; ++i) M.nobs_field[i] = nobs[i];
  const int nl = k * (k - 1) / 2;
  if (d->param == ADELIA_PARAM_UNIVARIATE) {
    M.d = 4;
    M.idx_prec[0] = 0; M.idx_range[0] = 1; M.idx_temporal[0] = 2; M.idx_tau[0] = 3;
    M.role_kind[0] = ROLE_COUPLING; M.role_idx[0] = 0;
    M.role_kind[1] = ROLE_RANGE; M.role_idx[1] = 0;
    M.role_kind[2] = ROLE_TEMPORAL; M.role_idx[2] = 0;
    M.role_kind[3] = ROLE_TAU; M.role_idx[3] = 0;
  } else {
    M.d = 4 * k + nl;
    for (int i = 0; i < k; ++i) {
      M.idx_range[i] = i; M.role_kind[i] = ROLE_RANGE; M.role_idx[i] = i;
      M.idx_temporal[i] = k + i; M.role_kind[k + i] = ROLE_TEMPORAL; M.role_idx[k + i] = i;
      M.idx_prec[i] = 2 * k + i; M.role_kind[2 * k + i] = ROLE_COUPLING; M.role_idx[2 * k + i] = i;
      M.idx_tau[i] = 3 * k + nl + i;
      M.role_kind[3 * k + nl + i] = ROLE_TAU; M.role_idx[3 * k + nl + i] = i;
    }
    for (int l = 0; l < nl; ++l) {
      M.idx_lambda[l] = 3 * k + l;
      M.role_kind[3 * k + l] = ROLE_COUPLING; M.role_idx[3 * k + l] = k + l;
    }
  }
  hipLaunchKernelGGL(yy_kernel, dim3(k), dim3(256), 0, 0, M, (double*)M.yy);
  m->Md = reinterpret_cast<const ModelDev*>(mem + offsets[15]);
  if (hipMemcpy(mem + offsets[15], &M, sizeof(ModelDev), hipMemcpyHostToDevice) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    hipFree(mem);
    delete m;
    return ADELIA_E_HIP;
  }
  m->split_sep = -1;
  if (full) {
    m->has_side = make_side(m->side, m->device);
    if (int r = build_split(ctx, d, m)) {
      inla_model_destroy(m);
      return r;
    }
  }
  *out = m;
  return 0;
}

int inla_model_create(adelia_ctx ctx, const inla_model_desc* d, inla_model* out) {
  set_last_error("");
  return model_create_impl(ctx, d, out, true);
}

// The halves of the two-sided split, created with the model (set-up time).  Half A is the model
// on blocks 0..sep (temporal entries and observations of those blocks); half B the model on
// blocks n-1, n-2, ..., sep (the temporal matrices read backwards; the sub-diagonal blocks are
// symmetric, so the reversed chain uses them as they are), whose last block -- the separator --
// has zero temporal coefficients and no observations, and whose fixed-effect prior precision is
// zero: its Schur complements then add to A's in the separator and the tip.  B has no
// hyperparameter prior (sigma = inf), so the two halves' gradients add up to the gradient.
static int build_split(adelia_ctx ctx, const inla_model_desc* d, inla_model m) {
  const int n = d->nt, k = d->k;
  if (n < 3) return 0;
  const int sep = (n - 1) / 2;
  const int ntA = sep + 1, ntB = n - sep;
  // half A: a prefix of the time steps and of the (time-sorted) observations
  inla_model_desc da = *d;
  da.nt = ntA;
  int oA = 0;
  while (oA < d->n_obs && d->obs_t[oA] <= sep) ++oA;
  da.n_obs = oA;
  // half B: reversed time, its observations re-sorted by (local time, field)
  std::vector<double> tdiag[3], toff[3];
  const double* diags[3] = {d->m0_diag, d->m1_diag, d->m2_diag};
  const double* offs[3] = {d->m0_off, d->m1_off, d->m2_off};
  for (int r = 0; r < 3; ++r) {
    tdiag[r].assign(ntB, 0.0);
    toff[r].assign(std::max(1, ntB - 1), 0.0);
    for (int t = 0; t < ntB - 1; ++t) {
      tdiag[r][t] = diags[r][n - 1 - t];
      toff[r][t] = offs[r][n - 2 - t];
    }
  }
  std::vector<int> ord;
  for (int o = oA; o < d->n_obs; ++o) ord.push_back(o);
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
    const int tx = n - 1 - d->obs_t[x], ty = n - 1 - d->obs_t[y];
    return tx != ty ? tx < ty : d->obs_field[x] < d->obs_field[y];
  });
  const int nB = (int)ord.size(), a = d->a;
  std::vector<int32_t> bt(nB), bf(nB), bnode(4 * (size_t)nB);
  std::vector<double> bw(4 * (size_t)nB), bX((size_t)nB * a), by(nB);
  for (int i = 0; i < nB; ++i) {
    const int o = ord[i];
    bt[i] = n - 1 - d->obs_t[o];
    bf[i] = d->obs_field[o];
    for (int q = 0; q < 4; ++q) {
      bnode[4 * i + q] = d->obs_node[4 * o + q];
      bw[4 * i + q] = d->obs_w[4 * o + q];
    }
    for (int c = 0; c < a; ++c) bX[(size_t)i * a + c] = d->X[(size_t)o * a + c];
    by[i] = d->y[o];
  }
  inla_model_desc db = *d;
  db.nt = ntB;
  db.m0_diag = tdiag[0].data(); db.m0_off = toff[0].data();
  db.m1_diag = tdiag[1].data(); db.m1_off = toff[1].data();
  db.m2_diag = tdiag[2].data(); db.m2_off = toff[2].data();
  db.n_obs = nB;
  db.obs_t = bt.data(); db.obs_field = bf.data(); db.obs_node = bnode.data();
  db.obs_w = bw.data(); db.X = bX.data(); db.y = by.data();
  if (int r = model_create_impl(ctx, &da, &m->half[0], false)) return r;
  if (int r = model_create_impl(ctx, &db, &m->half[1], false)) return r;
  ModelDev& MB = m->half[1]->M;
  MB.tip = 0.0;
  MB.sigma = INFINITY;
  (void)k;
  char* mem = nullptr;
  const size_t bytes = align_up(2 * sizeof(ModelDev)) + 256;
  if (hipMalloc(&mem, bytes) != hipSuccess) return ADELIA_E_HIP;
  m->half_dev = reinterpret_cast<ModelDev*>(mem);
  m->zn_split = reinterpret_cast<int32_t*>(mem + align_up(2 * sizeof(ModelDev)));
  const int32_t zn[4] = {sep, sep, ntB - 1, ntB - 1};
  ModelDev both[2] = {m->half[0]->M, MB};
  if (hipMemcpy(m->half_dev, both, sizeof(both), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m->zn_split, zn, sizeof(zn), hipMemcpyHostToDevice) != hipSuccess) {
    hipFree(mem);
    m->half_dev = nullptr;
    return ADELIA_E_HIP;
  }
  m->Mh = m->half[0]->M;
  m->Mh.nt = std::max(ntA, ntB);
  m->Mh.n_obs = std::max(m->half[0]->M.n_obs, MB.n_obs);
  m->Mh.nch_obs = std::max(m->half[0]->M.nch_obs, MB.nch_obs);
  m->Mh.nch_resid = std::max(m->half[0]->M.nch_resid, MB.nch_resid);
  m->Mr = m->M;
  m->Mr.nt = 1;
  m->split_sep = sep;
  return 0;
}

int inla_model_destroy(inla_model m) {
  if (!m) return 0;
  if (m->has_side) free_side(m->side);
  for (inla_model h : m->half) inla_model_destroy(h);
  if (m->half_dev) hipFree(m->half_dev);
  hipFree(m->dev_mem);
  delete m;
  return 0;
}

int inla_model_dim(inla_model m) { return m ? m->M.d : 0; }

size_t inla_workspace_bytes(inla_model m, int batch, int mode) {
  if (!m || batch < 1 || batch > 32767) return 0;
  if (mode == ADELIA_MODE_OBJECTIVE_SPLIT || mode == ADELIA_MODE_GRAD_SPLIT)
    return (batch == 1 && m->split_sep >= 0)
               ? split_layout(m, mode == ADELIA_MODE_GRAD_SPLIT, nullptr).bytes
               : 0;
  if (mode != ADELIA_MODE_OBJECTIVE && mode != ADELIA_MODE_GRAD && mode != ADELIA_MODE_GRAD_CARRY)
    return 0;
  return layout(m->M, batch, mode != ADELIA_MODE_OBJECTIVE, nullptr,
                mode == ADELIA_MODE_GRAD_CARRY).bytes;
}

int inla_objective(inla_model m, const double* theta, int32_t batch, double* f, int32_t* info,
                   void* ws, size_t ws_bytes, int flags, void* stream) {
  if (!m) return -1;
  if (!theta || !aligned(theta, 8)) return -2;
  if (batch < 1 || batch > 32767) return -3;
  if (!f || !aligned(f, 8)) return -4;
  if (!info || !aligned(info, 4)) return -5;
  if (!ws || !aligned(ws, 256)) return -6;
  if (flags & ~(ADELIA_SAVE_FACTORS | ADELIA_SPLIT)) return -8;
  const bool save = flags & ADELIA_SAVE_FACTORS;
  if (save && batch != 1) return -3;
  if (flags & ADELIA_SPLIT) {
    if (save) return -8;
    if (batch != 1) return -3;
    if (m->split_sep < 0) return ADELIA_E_UNSUPPORTED;
    const SplitWs sw = split_layout(m, false, reinterpret_cast<char*>(ws));
    if (ws_bytes < sw.bytes) return ADELIA_E_WORKSPACE;
    if (m->saved_ws == ws) m->saved_ws = nullptr;
    return run_split(m, sw, theta, f, nullptr, info, (hipStream_t)stream);
  }
  InlaWs w = layout(m->M, batch, save, reinterpret_cast<char*>(ws));
  if (ws_bytes < w.bytes) return ADELIA_E_WORKSPACE;
  if (int r = capture_guard((hipStream_t)stream,
                            launches_per_pass(m->M, m->has_side ? &m->side : nullptr, batch, save)))
    return r;
  m->saved_ws = save ? ws : (m->saved_ws == ws ? nullptr : m->saved_ws);
  return run_objective(eval_of(m), w, theta, f, info, (hipStream_t)stream,
                       m->has_side ? &m->side : nullptr);
}

int inla_grad(inla_model m, const double* theta, double* f, double* grad, int32_t* info, void* ws,
              size_t ws_bytes, int flags, void* stream) {
  if (!m) return -1;
  if (!theta || !aligned(theta, 8)) return -2;
  if (!f || !aligned(f, 8)) return -3;
  if (!grad || !aligned(grad, 8)) return -4;
  if (!info || !aligned(info, 4)) return -5;
  if (!ws || !aligned(ws, 256)) return -6;
  if (flags & ~(ADELIA_REUSE_FACTORS | ADELIA_CARRY_ONLY | ADELIA_SPLIT)) return -8;
  const bool carry = flags & ADELIA_CARRY_ONLY;
  if (carry && (flags & ADELIA_REUSE_FACTORS)) return -8;
  if (flags & ADELIA_SPLIT) {
    if (flags & (ADELIA_REUSE_FACTORS | ADELIA_CARRY_ONLY)) return -8;
    if (m->split_sep < 0) return ADELIA_E_UNSUPPORTED;
    const SplitWs sw = split_layout(m, true, reinterpret_cast<char*>(ws));
    if (ws_bytes < sw.bytes) return ADELIA_E_WORKSPACE;
    if (m->saved_ws == ws) m->saved_ws = nullptr;
    return run_split(m, sw, theta, f, grad, info, (hipStream_t)stream);
  }
  InlaWs w = layout(m->M, 1, true, reinterpret_cast<char*>(ws), carry);
  if (ws_bytes < w.bytes) return ADELIA_E_WORKSPACE;
  if ((flags & ADELIA_REUSE_FACTORS) && m->saved_ws != ws) return ADELIA_E_STATE;
  if (m->saved_ws == ws) m->saved_ws = nullptr;
  hipStream_t s = (hipStream_t)stream;
  if (!(flags & ADELIA_REUSE_FACTORS)) {
    int r = run_forward(eval_of(m), w, theta, s, m->has_side ? &m->side : nullptr);
    if (r) return r;
  }
  return run_backward(eval_of(m), w, theta, f, grad, info, nullptr, s,
                      m->has_side ? &m->side : nullptr);
}

int inla_grad_batched(inla_model m, const double* theta, int32_t batch, double* f, double* grad,
                      int32_t* info, void* ws, size_t ws_bytes, void* stream) {
  if (!m) return -1;
  if (!theta || !aligned(theta, 8)) return -2;
  if (batch < 1 || batch > 32767) return -3;
  if (!f || !aligned(f, 8)) return -4;
  if (!grad || !aligned(grad, 8)) return -5;
  if (!info || !aligned(info, 4)) return -6;
  if (!ws || !aligned(ws, 256)) return -7;
  InlaWs w = layout(m->M, batch, true, reinterpret_cast<char*>(ws));
  if (ws_bytes < w.bytes) return ADELIA_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  if (int r = capture_guard(s, launches_per_pass(m->M, m->has_side ? &m->side : nullptr, batch,
                                                 true)))
    return r;
  if (m->saved_ws == ws) m->saved_ws = nullptr;
  int r = run_forward(eval_of(m), w, theta, s, m->has_side ? &m->side : nullptr);
  if (r) return r;
  return run_backward(eval_of(m), w, theta, f, grad, info, nullptr, s,
                      m->has_side ? &m->side : nullptr);
}

int inla_grad_terms(inla_model m, const double* theta, double* terms, int32_t* info, void* ws,
                    size_t ws_bytes, int flags, void* stream) {
  if (!m) return -1;
  if (!theta || !aligned(theta, 8)) return -2;
  if (!terms || !aligned(terms, 8)) return -3;
  if (!info || !aligned(info, 4)) return -4;
  if (!ws || !aligned(ws, 256)) return -5;
  if (flags & ~(ADELIA_REUSE_FACTORS | ADELIA_CARRY_ONLY)) return -7;
  const bool carry = flags & ADELIA_CARRY_ONLY;
  if (carry && (flags & ADELIA_REUSE_FACTORS)) return -7;
  InlaWs w = layout(m->M, 1, true, reinterpret_cast<char*>(ws), carry);
  if (ws_bytes < w.bytes) return ADELIA_E_WORKSPACE;
  if ((flags & ADELIA_REUSE_FACTORS) && m->saved_ws != ws) return ADELIA_E_STATE;
  if (m->saved_ws == ws) m->saved_ws = nullptr;
  hipStream_t s = (hipStream_t)stream;
  if (!(flags & ADELIA_REUSE_FACTORS)) {
    int r = run_forward(eval_of(m), w, theta, s, m->has_side ? &m->side : nullptr);
    if (r) return r;
  }
  const int d = m->M.d;
  return run_backward(eval_of(m), w, theta, terms, terms + 5 + 5 * d, info, terms, s,
                      m->has_side ? &m->side : nullptr);
}

int inla_fd_grad(inla_model m, const double* theta, double h, int32_t max_batch, double* f,
                 double* grad, int32_t* info, void* ws, size_t ws_bytes, void* stream) {
  if (!m) return -1;
  if (!theta || !aligned(theta, 8)) return -2;
  if (!(h > 0.0)) return -3;
  if (max_batch < 1 || max_batch > 32767) return -4;
  if (!f || !aligned(f, 8)) return -5;
  if (!grad || !aligned(grad, 8)) return -6;
  if (!info || !aligned(info, 4)) return -7;
  if (!ws || !aligned(ws, 256)) return -8;
  const int d = m->M.d, npts = 2 * d + 1;
  const int bmax = std::min<int>(max_batch, npts);
  InlaWs w = layout(m->M, bmax, false, reinterpret_cast<char*>(ws));
  if (ws_bytes < w.bytes) return ADELIA_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  if (int r = capture_guard(s, planned_passes(m, npts, bmax, false))) return r;
  if (m->saved_ws == ws) m->saved_ws = nullptr;
  hipLaunchKernelGGL(stencil_kernel, dim3((npts * d + 255) / 256), dim3(256), 0, s, theta, d, h,
                     w.Th);
  if (!LAUNCH_OK()) return ADELIA_E_HIP;
  for (int p0 = 0; p0 < npts; p0 += bmax) {
    const int bs = std::min(bmax, npts - p0);
    // a smaller last sub-batch uses a prefix of the same workspace; the stencil scratch sits
    // at a fixed place in front of it
    InlaWs wb = layout(m->M, bs, false, reinterpret_cast<char*>(ws));
    int r = run_objective(eval_of(m), wb, w.Th + (long long)p0 * d, w.fv + p0, info + p0, s,
                          m->has_side ? &m->side : nullptr);
    if (r) return r;
  }
  hipLaunchKernelGGL(fd_kernel, dim3((d + 63) / 64), dim3(64), 0, s, w.fv, d, h, f, grad);
  return LAUNCH_OK() ? 0 : ADELIA_E_HIP;
}

int inla_hessian(inla_model m, const double* theta, double h, int32_t max_batch, double* f,
                 double* grad, double* H, int32_t* info, void* ws, size_t ws_bytes, void* stream) {
  if (!m) return -1;
  if (!theta || !aligned(theta, 8)) return -2;
  if (!(h > 0.0)) return -3;
  if (max_batch < 1 || max_batch > 32767) return -4;
  if (!f || !aligned(f, 8)) return -5;
  if (!grad || !aligned(grad, 8)) return -6;
  if (!H || !aligned(H, 8)) return -7;
  if (!info || !aligned(info, 4)) return -8;
  if (!ws || !aligned(ws, 256)) return -9;
  const int d = m->M.d, npts = 2 * d + 1;
  const int bmax = std::min<int>(max_batch, npts);
  InlaWs w = layout(m->M, bmax, true, reinterpret_cast<char*>(ws));
  if (ws_bytes < w.bytes) return ADELIA_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  if (int r = capture_guard(s, planned_passes(m, npts, bmax, true))) return r;
  if (m->saved_ws == ws) m->saved_ws = nullptr;
  hipLaunchKernelGGL(stencil_kernel, dim3((npts * d + 255) / 256), dim3(256), 0, s, theta, d, h,
                     w.Th);
  if (!LAUNCH_OK()) return ADELIA_E_HIP;
  // exact gradients of the points, `bmax` at a time (a smaller last sub-batch uses a prefix of
  // the same workspace; the stencil scratch sits at a fixed place in front of it)
  for (int p0 = 0; p0 < npts; p0 += bmax) {
    const int bs = std::min(bmax, npts - p0);
    InlaWs wb = layout(m->M, bs, true, reinterpret_cast<char*>(ws));
    const double* th = w.Th + (long long)p0 * d;
    int r = run_forward(eval_of(m), wb, th, s, m->has_side ? &m->side : nullptr);
    if (r) return r;
    r = run_backward(eval_of(m), wb, th, w.fv + p0, w.gv + (long long)p0 * d, info + p0, nullptr, s,
                     m->has_side ? &m->side : nullptr);
    if (r) return r;
  }
  hipLaunchKernelGGL(grad_hessian_kernel, dim3((d * d + 63) / 64), dim3(64), 0, s, w.fv, w.gv, d,
                     h, f, grad, H);
  return LAUNCH_OK() ? 0 : ADELIA_E_HIP;
}

int inla_fd_hessian(inla_model m, const double* theta, double h, int32_t max_batch, double* f,
                    double* H, int32_t* info, void* ws, size_t ws_bytes, void* stream) {
  if (!m) return -1;
  if (!theta || !aligned(theta, 8)) return -2;
  if (!(h > 0.0)) return -3;
  if (max_batch < 1 || max_batch > 32767) return -4;
  if (!f || !aligned(f, 8)) return -5;
  if (!H || !aligned(H, 8)) return -6;
  if (!info || !aligned(info, 4)) return -7;
  if (!ws || !aligned(ws, 256)) return -8;
  const int d = m->M.d, npts = 2 * d * d + 1;
  const int bmax = std::min<int>(max_batch, npts);
  InlaWs w = layout(m->M, bmax, false, reinterpret_cast<char*>(ws));
  if (ws_bytes < w.bytes) return ADELIA_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  if (int r = capture_guard(s, planned_passes(m, npts, bmax, false))) return r;
  if (m->saved_ws == ws) m->saved_ws = nullptr;
  hipLaunchKernelGGL(hess_stencil_kernel, dim3((npts * d + 255) / 256), dim3(256), 0, s, theta, d,
                     h, w.Th);
  if (!LAUNCH_OK()) return ADELIA_E_HIP;
  for (int p0 = 0; p0 < npts; p0 += bmax) {
    const int bs = std::min(bmax, npts - p0);
    InlaWs wb = layout(m->M, bs, false, reinterpret_cast<char*>(ws));
    int r = run_objective(eval_of(m), wb, w.Th + (long long)p0 * d, w.fv + p0, info + p0, s,
                          m->has_side ? &m->side : nullptr);
    if (r) return r;
  }
  hipLaunchKernelGGL(fd_hessian_kernel, dim3((d * d + 63) / 64), dim3(64), 0, s, w.fv, d, h, f,
                     H);
  return LAUNCH_OK() ? 0 : ADELIA_E_HIP;
}

int inla_batch_create(adelia_ctx ctx, int count, const inla_model* models, inla_batch* out) {
  set_last_error("");
  if (!ctx) return -1;
  if (count < 1 || count > 32767) return -2;
  if (!models) return -3;
  if (!out) return -4;
  for (int i = 0; i < count; ++i)
    if (!models[i] || models[i]->device != ctx->device) return -3;
  const inla_model m0 = models[0];
  for (int i = 1; i < count; ++i) {
    const inla_model m = models[i];
    if (m->param != m0->param || m->M.k != m0->M.k || m->M.d != m0->M.d)
      return fail("batched models need the same parameterisation, k and d");
  }
  // groups by block size, members in batch order
  std::map<int, std::vector<int>> by_b;
  for (int i = 0; i < count; ++i) by_b[models[i]->M.b].push_back(i);
  std::vector<BatchGroup> groups;
  size_t total = 0;
  std::vector<size_t> xoff;  // per instance: offset of its padded X (or SIZE_MAX)
  xoff.assign(count, SIZE_MAX);
  std::vector<size_t> goff;  // per group: offset of its Mv, zn, idx arrays
  for (auto& kv : by_b) {
    BatchGroup g;
    g.members = kv.second;
    g.Mh = models[g.members[0]]->M;
    for (int q : g.members) {
      const ModelDev& M = models[q]->M;
      if (M.ns != g.Mh.ns || M.nch_rows != g.Mh.nch_rows)
        return fail("batched models of one block size need the same spatial size");
      g.Mh.nt = std::max(g.Mh.nt, M.nt);
      g.Mh.a = std::max(g.Mh.a, M.a);
      g.Mh.nch_obs = std::max(g.Mh.nch_obs, M.nch_obs);
      g.Mh.nch_resid = std::max(g.Mh.nch_resid, M.nch_resid);
      g.Mh.n_obs = std::max(g.Mh.n_obs, M.n_obs);
      g.Mh.wband_w = std::max(g.Mh.wband_w, M.wband_w);
      g.Mh.wdeg = std::max(g.Mh.wdeg, M.wdeg);
    }
    if ((long long)g.Mh.b * g.Mh.nt + g.Mh.a > INT_MAX) return fail("batch group too large");
    goff.push_back(total);
    const int ng = (int)g.members.size();
    total = align_up(total + (size_t)ng * sizeof(ModelDev));
    total = align_up(total + (size_t)2 * ng * 4);
    total = align_up(total + (size_t)ng * 4);
    for (int q : g.members) {
      const ModelDev& M = models[q]->M;
      if (M.a < g.Mh.a && M.n_obs > 0) {
        xoff[q] = total;
        total = align_up(total + (size_t)M.n_obs * g.Mh.a * 8);
      }
    }
    groups.push_back(std::move(g));
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return ADELIA_E_HIP;
  char* mem = nullptr;
  if (hipMalloc(&mem, std::max<size_t>(total, 256)) != hipSuccess) return ADELIA_E_HIP;
  inla_batch B = new inla_batch_s();
  B->device = ctx->device;
  B->d = m0->M.d;
  B->count = count;
  B->dev_mem = mem;
  bool ok = true;
  for (size_t gi = 0; gi < groups.size() && ok; ++gi) {
    BatchGroup& g = groups[gi];
    const int ng = (int)g.members.size();
    size_t off = goff[gi];
    g.Mv = reinterpret_cast<ModelDev*>(mem + off);
    off = align_up(off + (size_t)ng * sizeof(ModelDev));
    g.zn = reinterpret_cast<int32_t*>(mem + off);
    off = align_up(off + (size_t)2 * ng * 4);
    g.idx = reinterpret_cast<int32_t*>(mem + off);
    std::vector<ModelDev> mv;
    std::vector<int32_t> zn, idx;
    for (int q : g.members) {
      ModelDev M = models[q]->M;
      if (xoff[q] != SIZE_MAX) {
        double* Xp = reinterpret_cast<double*>(mem + xoff[q]);
        const long long cnt = (long long)M.n_obs * g.Mh.a;
        hipLaunchKernelGGL(pad_cols_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, 0,
                           M.X, M.n_obs, M.a, g.Mh.a, Xp);
        M.X = Xp;
      }
      M.a = g.Mh.a;
      mv.push_back(M);
      zn.push_back(M.nt);
      zn.push_back(M.nt);
      idx.push_back(q);
    }
    ok = hipMemcpy(g.Mv, mv.data(), mv.size() * sizeof(ModelDev), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(g.zn, zn.data(), zn.size() * 4, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(g.idx, idx.data(), idx.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
  }
  if (!ok || hipDeviceSynchronize() != hipSuccess) {
    hipFree(mem);
    delete B;
    return ADELIA_E_HIP;
  }
  B->groups = std::move(groups);
  B->has_side = make_side(B->side, B->device);
  *out = B;
  return 0;
}

int inla_batch_destroy(inla_batch B) {
  if (!B) return 0;
  if (B->has_side) free_side(B->side);
  hipFree(B->dev_mem);
  delete B;
  return 0;
}

int inla_batch_groups(inla_batch B) { return B ? (int)B->groups.size() : 0; }

size_t inla_batch_workspace_bytes(inla_batch B, int mode) {
  if (!B) return 0;
  if (mode != ADELIA_MODE_OBJECTIVE && mode != ADELIA_MODE_GRAD) return 0;
  return batch_ws_bytes(B, mode == ADELIA_MODE_GRAD);
}

int inla_batch_objective(inla_batch B, const double* theta, double* f, int32_t* info, void* ws,
                         size_t ws_bytes, void* stream) {
  if (!B) return -1;
  if (!theta || !aligned(theta, 8)) return -2;
  if (!f || !aligned(f, 8)) return -3;
  if (!info || !aligned(info, 4)) return -4;
  if (!ws || !aligned(ws, 256)) return -5;
  if (ws_bytes < batch_ws_bytes(B, false)) return ADELIA_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  if (int r = capture_guard(s, batch_launches(B, false))) return r;
  return batch_eval(B, theta, f, nullptr, info, ws, s, false);
}

int inla_batch_grad(inla_batch B, const double* theta, double* f, double* grad, int32_t* info,
                    void* ws, size_t ws_bytes, void* stream) {
  if (!B) return -1;
  if (!theta || !aligned(theta, 8)) return -2;
  if (!f || !aligned(f, 8)) return -3;
  if (!grad || !aligned(grad, 8)) return -4;
  if (!info || !aligned(info, 4)) return -5;
  if (!ws || !aligned(ws, 256)) return -6;
  if (ws_bytes < batch_ws_bytes(B, true)) return ADELIA_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  if (int r = capture_guard(s, batch_launches(B, true))) return r;
  return batch_eval(B, theta, f, grad, info, ws, s, true);
}

int inla_autotune(inla_model m, const double* theta, int32_t batch, int mode, int reps, void* ws,
                  size_t ws_bytes, void* stream, int32_t* changed) {
  if (!m) return -1;
  if (!theta || !aligned(theta, 8)) return -2;
  const int d = m->M.d;
  if (batch < 1 || batch > 2 * d + 1) return -3;
  if (mode != ADELIA_MODE_OBJECTIVE && mode != ADELIA_MODE_GRAD) return -4;
  if (reps < 1 || reps > 100) return -5;
  if (!ws || !aligned(ws, 256)) return -6;
  if (!changed) return -9;
  const bool grad = mode == ADELIA_MODE_GRAD;
  InlaWs w = layout(m->M, batch, grad, reinterpret_cast<char*>(ws));
  if (ws_bytes < w.bytes) return ADELIA_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess || st != hipStreamCaptureStatusNone)
    return ADELIA_E_UNSUPPORTED;  // it synchronises: set-up time only
  if (m->saved_ws == ws) m->saved_ws = nullptr;
  const SideRes* side = m->has_side ? &m->side : nullptr;
  // the results land in the workspace's stencil scratch (room for 2d + 1 points)
  auto eval = [&]() -> int {
    if (!grad) return run_objective(eval_of(m), w, theta, w.fv, w.finfo, s, side);
    int r = run_forward(eval_of(m), w, theta, s, side);
    return r ? r : run_backward(eval_of(m), w, theta, w.fv, w.gv, w.finfo, nullptr, s, side);
  };
  *changed = 0;
  int c = 0;
  const int r = tune_block_size(m->M.b, eval, reps, s, &c);
  *changed = c;
  if (r) return r;
  tune_save_env();
  return 0;
}

int inla_batch_autotune(inla_batch B, const double* theta, int mode, int reps, void* ws,
                        size_t ws_bytes, void* stream, int32_t* changed) {
  if (!B) return -1;
  if (!theta || !aligned(theta, 8)) return -2;
  if (mode != ADELIA_MODE_OBJECTIVE && mode != ADELIA_MODE_GRAD) return -3;
  if (reps < 1 || reps > 100) return -4;
  if (!ws || !aligned(ws, 256)) return -5;
  if (!changed) return -8;
  const bool grad = mode == ADELIA_MODE_GRAD;
  if (ws_bytes < batch_ws_bytes(B, grad)) return ADELIA_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess || st != hipStreamCaptureStatusNone)
    return ADELIA_E_UNSUPPORTED;
  *changed = 0;
  int c = 0;
  for (int gi = 0; gi < (int)B->groups.size(); ++gi) {
    auto eval = [&]() -> int {
      return batch_eval(B, theta, nullptr, nullptr, nullptr, ws, s, grad, gi, gi + 1);
    };
    const int r = tune_block_size(B->groups[gi].Mh.b, eval, reps, s, &c);
    *changed = c;
    if (r) return r;
  }
  tune_save_env();
  return 0;
}

}  // extern "C"
