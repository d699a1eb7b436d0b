// Device code of the panel step (leaves, merges, row solves) is in panel_dev.h; the panel
// kernel and its host launcher are here.
#include "common.h"
#include "panel_dev.h"
#include "profile.h"
#include <algorithm>
#include <cmath>

namespace adelia {

using namespace panel_dev;

namespace {

__global__ __launch_bounds__(256) void potrf_panel_kernel(const PanelArgs P) {
  __shared__ PanelSmem sm;
  panel_body(P, blockIdx.x, gridDim.x, sm, blockIdx.z);
}

}  // namespace

int panel_workgroups(int b, int c0, int mT) {
  return (b - c0 + NB - 1) / NB + (mT + NB - 1) / NB;
}

double panel_flops(int b, int c0, int mT, int upd) {
  const double ww = (b - c0) < NB ? (b - c0) : NB;
  const double below = (double)(b - c0) - ww + mT;
  // with upd, the rank-64 update of the panel's columns (lower part of the diagonal tile and
  // every row below) is part of the launch
  const double updfl = (upd && c0 >= NB) ? 2.0 * NB * (ww * (ww + 1) / 2.0 + below * ww) : 0.0;
  return ww * ww * ww / 3.0 + below * ww * ww + updfl;
}

double panel_bytes(int b, int c0, int mT, int upd) {
  const double ww = (b - c0) < NB ? (b - c0) : NB;
  const double below = (double)(b - c0) - ww + mT;
  // the panel's columns read and written once (lower part of the diagonal tile and every row
  // below), the diagonal tile's inverse written, and with upd the previous panel's columns on
  // the same rows read
  const double cols = ww * (ww + 1) / 2.0 + below * ww;
  const double prev = (upd && c0 >= NB) ? (ww + below) * NB : 0.0;
  return 8.0 * (2.0 * cols + ww * ww + prev);
}

int launch_panel_diag(double* D, long long zD, double* G, long long zG, double* ldp,
                      long long zLd, int32_t* info, int32_t* cnt, const int32_t* zn, int step,
                      int b, int c0, long long gcol0, int upd, double* V, long long zV, int nz,
                      hipStream_t s) {
  if (!cnt) return -1;
  PanelArgs P{D, zD, G, zG, ldp, zLd, info, cnt, zn, step, b, c0, gcol0, nullptr, 0, 0, 0, upd,
              V, zV};
  const ProfToken t = prof_begin(s);
  hipLaunchKernelGGL(potrf_panel_kernel, dim3(1, 1, nz), dim3(256), 0, s, P);
  if (t.valid)
    prof_end(t, s, PK_PANEL, nz * panel_flops(std::min(b, c0 + NB), c0, 0, upd),
             nz * panel_bytes(std::min(b, c0 + NB), c0, 0, upd));
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_potrf_panel(double* D, long long zD, double* G, long long zG, double* ldp,
                       long long zLd, int32_t* info, int32_t* cnt, const int32_t* zn, int step,
                       int b, int c0, long long gcol0, double* T, long long zT, int ldT, int mT,
                       int upd, int nz, hipStream_t s) {
  if (!cnt) return -1;
  if (!T) mT = 0;
  if (mT < 0 || (mT > 0 && ldT < mT)) return -1;
  PanelArgs P{D, zD, G, zG, ldp, zLd, info, cnt, zn, step, b, c0, gcol0, T, zT, ldT, mT, upd};
  const int rows = panel_workgroups(b, c0, mT);
  const ProfToken t = prof_begin(s);
  hipLaunchKernelGGL(potrf_panel_kernel, dim3(rows, 1, nz), dim3(256), 0, s, P);
  if (t.valid)
    prof_end(t, s, PK_PANEL, nz * panel_flops(b, c0, mT, upd), nz * panel_bytes(b, c0, mT, upd));
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace adelia
