// One step of the look-ahead blocked Cholesky of a diagonal block as a single launch
// (Sec. III-A-1, Alg. 1, chol()): the workgroups of panel k+1 come first in the grid, so they
// are placed before any others, and the remaining workgroups apply panel k's rank-64 update to
// the columns from c0_k + 128 on (and to the rows of [B_i; C~_i] below them).  Panel k+1 applies
// panel k's update to its own columns itself, so the two parts touch disjoint columns: the
// update writes columns >= c0_{k+1} + 64 and reads those of panel k, which panel k+1 only reads.
// Consecutive steps run in stream order, with no events between them.
#include "common.h"
#include "gemm_dev.h"
#include "launchers.h"
#include "panel_dev.h"
#include "profile.h"

#include <climits>

namespace adelia {

namespace {

// the update part of a step computes two tiles of a row per workgroup (gemm_walk_pairs)
constexpr bool kStepPairs = true;

struct GemmSmem {
  double As[2][gemm_dev::BK][gemm_dev::LDS_ROW];
  double Bs[2][gemm_dev::BK][gemm_dev::LDS_ROW];
  double Bs1[2][gemm_dev::BK][gemm_dev::LDS_ROW];  // the second tile of a pair
};

union StepSmem {
  panel_dev::PanelSmem p;
  GemmSmem g;
};
static_assert(sizeof(GemmSmem) <= sizeof(panel_dev::PanelSmem),
              "the update's operand buffers fit in the panel's LDS");

// A one-dimensional grid: the panel workgroups of every chain first (npw per chain, the range
// padded to a multiple of 8), so that all of them are placed in the first round of
// workgroups, then ntw update workgroups per chain (ntw a multiple of 8, so that an update
// workgroup's index within its chain and within the grid fall on the same XCD).  pairs: the
// update's workgroups take two tiles of a row at once (gemm_walk_pairs; ntw covers units),
// else one tile each (gemm_walk).
__global__ __launch_bounds__(256) void panel_step_kernel(const panel_dev::PanelArgs P, int npw,
                                                         const GemmArgs U, int ntw, int pairs,
                                                         int nz) {
  static_assert(gemm_dev::NT == 256, "the panel and the tile GEMM share the workgroup shape");
  __shared__ StepSmem sm;
  const int bx = blockIdx.x;
  const int np = ((npw * nz + 7) & ~7);
  if (bx < np) {
    if (bx >= npw * nz) return;
    const int z = bx / npw;
    panel_dev::panel_body(P, bx - z * npw, npw, sm.p, z);
    return;
  }
  const int u = bx - np;
  const int z = u / ntw;
  if (U.zn && U.step >= U.zn[z]) return;  // chain z has no block at this step
  if (pairs)
    gemm_dev::gemm_walk_pairs(U, z, u - z * ntw, ntw, sm.g.As, sm.g.Bs, sm.g.Bs1);
  else
    gemm_dev::gemm_walk<true>(U, z, 0, true, u - z * ntw, ntw, sm.g.As, sm.g.Bs);
}

}  // namespace

int launch_panel_step(double* D, long long zD, double* G, long long zG, double* ldp,
                      long long zLd, int32_t* info, int32_t* cnt, const int32_t* zn, int step,
                      int b, int c0, long long gcol0, double* T, long long zT, int ldT, int mT,
                      int upd, int nz, const GemmArgs* U, int maxw, hipStream_t s) {
  long long tiles = 0, units = 0;
  if (U) {
    // one sub-problem, one phase, lower output (the trailing update)
    if (U->nph != 1 || U->omode == OUT_ALL || U->M != U->Mlast || U->N != U->Nlast ||
        U->M < U->N)
      return -1;
    const long long tM = (U->M + gemm_dev::BM - 1) / gemm_dev::BM;
    const long long tN = (U->N + gemm_dev::BN - 1) / gemm_dev::BN;
    tiles = U->N > 0 ? tN * (tN + 1) / 2 + (tM - tN) * tN : 0;
    units = U->N > 0 ? gemm_dev::pair_units((int)tM, (int)tN) : 0;
  }
  // tile pairs: the K range may not depend on the column, and B may not be triangular
  const bool pairs = U && kStepPairs && (U->ph[0].kmode == KR_FULL || U->ph[0].kmode == KR_LT_M1) &&
                     U->ph[0].triB == TRI_NONE;
  if (tiles == 0)
    return launch_potrf_panel(D, zD, G, zG, ldp, zLd, info, cnt, zn, step, b, c0, gcol0, T, zT,
                              ldT, mT, upd, nz, s);
  if (!cnt) return -1;
  if (!T) mT = 0;
  if (mT < 0 || (mT > 0 && ldT < mT) || nz > 65535) return -1;
  panel_dev::PanelArgs P{D, zD, G, zG, ldp, zLd, info, cnt, zn, step, b, c0, gcol0, T, zT, ldT,
                         mT, upd};
  const int npw = panel_workgroups(b, c0, mT);
  long long ntw = pairs ? units : tiles;
  if (maxw > 0 && ntw > maxw) ntw = maxw < 8 ? 8 : (maxw & ~7);
  ntw = (ntw + 7) & ~7LL;
  const long long grid = (((long long)npw * nz + 7) & ~7LL) + ntw * nz;
  if (grid > INT_MAX) return -1;
  const ProfToken t = prof_begin(s);
  hipLaunchKernelGGL(panel_step_kernel, dim3((unsigned)grid), dim3(256), 0, s, P, npw, *U,
                     (int)ntw, pairs ? 1 : 0, nz);
  if (t.valid)
    prof_end(t, s, PK_STEP, nz * panel_flops(b, c0, mT, upd) + gemm_flops(*U, 1) * nz,
             nz * panel_bytes(b, c0, mT, upd) + gemm_bytes(*U, 1) * nz);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace adelia
