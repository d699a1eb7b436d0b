// Launch wrappers implemented in panel.hip / step.hip / potrf.hip / util.hip (host side).
#pragma once
#include "common.h"

#define ADELIA_E_HIP_INTERNAL (-102)

namespace adelia {
// The diagonal tile of a panel alone (one workgroup per chain): L_kk, L_kk^-1, the log-diagonal
// partial and the pivot check, and with upd and V the product V = L_kk^-1 Q (panel_dev.h).
int launch_panel_diag(double* D, long long zD, double* G, long long zG, double* ldp,
                      long long zLd, int32_t* info, int32_t* cnt, const int32_t* zn, int step,
                      int b, int c0, long long gcol0, int upd, double* V, long long zV, int nz,
                      hipStream_t s);
int launch_potrf_panel(double* D, long long zD, double* G, long long zG, double* ldp,
                       long long zLd, int32_t* info, int32_t* cnt, const int32_t* zn, int step,
                       int b, int c0, long long gcol0, double* T, long long zT, int ldT, int mT,
                       int upd, int nz, hipStream_t s);
// Workgroups of one panel launch per chain, and its algorithmic flops and compulsory HBM bytes
// per chain.
int panel_workgroups(int b, int c0, int mT);
double panel_flops(int b, int c0, int mT, int upd);
double panel_bytes(int b, int c0, int mT, int upd);
// Panel launch fused with the trailing update U of the previous panel (step.hip); U == nullptr
// or an empty U: the panel alone.  At most maxw workgroups (0: one per tile) walk U's tiles.
int launch_panel_step(double* D, long long zD, double* G, long long zG, double* ldp,
                      long long zLd, int32_t* info, int32_t* cnt, const int32_t* zn, int step,
                      int b, int c0, long long gcol0, double* T, long long zT, int ldT, int mT,
                      int upd, int nz, const GemmArgs* U, int maxw, hipStream_t s);
int launch_tip(double* T, long long zT, int a, int ap, double* ldp, long long zLd, int32_t* info,
               long long gcol0, double* zsq, double* ZT, long long zZT, double* xT,
               long long zXT, int nz, hipStream_t s);
int launch_gemv_n(const double* A, long long ld, long long zA, const double* x, long long zx,
                  long long incx, const double* y0, long long zy0, long long incy0, double* y,
                  long long zy, long long incy, int M, int K, int lowerA, double alpha,
                  double beta, int nz, hipStream_t s);
int launch_tri_small(const double* L, long long ld, long long zL, double* v, long long zv, int a,
                     int trans, int nz, hipStream_t s);
int launch_logdiag(const double* L, int b, long long ld, long long bs, int nblk, double* part,
                   long long zL, long long zp, int nz, hipStream_t s);
int launch_fill_strided(double* p, long long stride, int count, double v, hipStream_t s);
// C = alpha (A1 B1 + A2 B2) + beta C for m <= kSkinnyRows rows (util.hip); A2 may be null
constexpr int kSkinnyRows = 8, kSkinnyCols = 8;
struct Skinny {
  int m, N, K1, K2;
  const double* A1; long long lda1, zA1;
  const double* B1; long long ldb1, zB1;
  const double* A2; long long lda2, zA2;
  const double* B2; long long ldb2, zB2;
  double* C; long long ldc, zC;
  double alpha, beta;
  const int32_t* zn; int step;  // chain z takes part only while step < zn[z] (zn may be null)
  int zdiv;    // > 0: grid.z runs over (chain, block) pairs as in GemmArgs::zdiv
  int lowerB;  // B1 lower triangular: B1(k, n) = 0 for k < n is neither read nor summed
};
int launch_skinny(const Skinny& g, int nz, hipStream_t s);
}  // namespace adelia
