// Device-resident INLA model description (passed by value to the kernels).
#pragma once
#include "common.h"

namespace adelia {

enum Role { ROLE_RANGE = 0, ROLE_TEMPORAL = 1, ROLE_COUPLING = 2, ROLE_TAU = 3 };

constexpr int kTraceRows = 64;  // pattern rows per trace workgroup (four lanes per row)
constexpr int kTraceObs = 16;   // observations per trace workgroup (sixteen lanes each)
constexpr int kResidObs = 1024;  // observations per residual workgroup

struct ModelDev {
  int k, ns, nt, a, b, n_obs, d, nnz;
  // the traces of one block are summed in slices (kTraceRows pattern rows, kTraceObs
  // observations per workgroup) whose partial sums are added in slice order at the end
  int nch_rows, nch_obs;
  int nch_resid;  // slices of kResidObs observations of the data residual
  double sigma, tip;
  const int32_t* uptr;   // union pattern of c0, g1, g2 (CSR, ns + 1)
  const int32_t* uidx;   // nnz
  const double* uval;    // 3 * nnz: value of c0, g1, g2 on the union pattern
  const double* tm;      // 3 x (2 nt - 1): diagonal then sub-diagonal of M0, M1, M2
  const int32_t* obs_t;
  const int32_t* obs_f;
  const int32_t* obs_node;  // n_obs x 4
  const double* obs_w;      // n_obs x 4
  const double* X;          // n_obs x a
  const double* y;
  const int32_t* obs_off;   // nt*k + 1: first observation of (t, field)
  const int32_t* colptr;    // nt*b + 1: observation entries touching (t, column)
  const int32_t* col_o;
  const int32_t* col_e;
  const double* yy;         // k: sum of y^2 per field
  // the banded W_t product: per tile of kWRows pattern rows, the range [lo, hi) of pattern
  // columns its rows touch; the widest range and the most entries in one pattern row
  const int32_t* wband;
  int wband_w, wdeg;
  int nobs_field[kMaxFields];
  int idx_range[kMaxFields], idx_temporal[kMaxFields], idx_prec[kMaxFields];
  int idx_lambda[kMaxFields * (kMaxFields - 1) / 2], idx_tau[kMaxFields];
  int role_kind[kMaxTheta], role_idx[kMaxTheta];
};

// The model(s) a launch reads: one model for every theta point (each == 0: v[0]), or one per
// point (each == 1: point p evaluates model v[p], an uneven batch of instances that share the
// block size and arrow width; chain z belongs to point z / 2).  The kernels take their model
// as a copy from device memory, so one launch can cover instances of different models.
struct Models {
  const ModelDev* v;
  int each;
};
__device__ __forceinline__ ModelDev model_at(const Models& ms, int p) {
  return ms.v[ms.each ? p : 0];
}

__global__ void param_kernel(const Models Ms, const double* theta, double* phi, double* dphi,
                             double* tau);
__global__ void assemble_blocks_kernel(const Models Ms, int td, int tb, double* D, long long zD,
                                       double* B, long long zB, long long ldB, const double* phi,
                                       const double* tau);
__global__ void assemble_arrow_kernel(const Models Ms, double* C, long long zC, long long nb,
                                      int ap,
                                      const double* tau);
__global__ void assemble_tip_kernel(const Models Ms, double* T, long long zT, int ap,
                                    const double* tau);
__global__ void trace_kernel(const Models Ms, int j, const double* ZD, long long zZD,
                             const double* ZB, long long zZB, const double* ZC, long long zZC,
                             const double* ZT, long long zZT, double* TD, double* TB, double* O,
                             long long zTr, long long zO);
__global__ void phaseb_kernel(const Models Ms, const double* x, long long zxp, double* qD,
                              double* qB, long long zq);
__global__ void resid_kernel(const Models Ms, const double* x, long long zxp, int nlay,
                             double* resid, long long zr);
__global__ void objective_kernel(const Models Ms, const double* theta, int batch,
                                 const double* tau, const double* ld, const double* zsq,
                                 const int32_t* info, double* f, int32_t* info_out);
__global__ void grad_kernel(const Models Ms, const double* theta, const double* dphi,
                            const double* tau, const double* TD, const double* TB, long long zTr,
                            const double* O, long long zO, const double* qD, const double* qB,
                            long long zq, const double* resid, long long zr, const double* ld,
                            const double* zsq, const double* ZTc, long long zZT,
                            const int32_t* info, double* f, double* grad, int32_t* info_out,
                            double* terms);
__global__ void yy_kernel(const ModelDev M, double* yy);
__global__ void split_merge_kernel(const double* D, long long zD, long long sD, int slotsD,
                                   const double* C, long long zC, long long sC, const double* T,
                                   long long zT, const int32_t* zn, int b, int ap, double* Dr,
                                   long long zDr, double* Cr, long long zCr, double* Tr,
                                   long long zTr);
__global__ void split_seed_kernel(const double* ZDr, long long zZDr, const double* ZCr,
                                  long long zZCr, const double* ZTr, long long zZTr,
                                  const double* xr, long long zxr, const double* xTr,
                                  long long zxTr, int b, int a, const int32_t* zn, int slotsZD,
                                  double* ZD, long long zZD, double* ZC, long long zZC,
                                  double* ZT, long long zZT, double* x, long long zx, double* xT,
                                  long long zxT);
__global__ void split_combine_kernel(const Models Ms, const double* theta, const double* tau,
                                     const double* ldh, const double* ldr, const double* zsqr,
                                     const int32_t* infh, const int32_t* infr, const double* gv,
                                     const int32_t* ginfo, double* f, double* grad,
                                     int32_t* info);
__global__ void stencil_kernel(const double* theta, int d, double h, double* Th);
__global__ void fd_kernel(const double* fv, int d, double h, double* f, double* grad);
__global__ void hess_stencil_kernel(const double* theta, int d, double h, double* Th);
constexpr int kWBatch = 8;  // columns of W_t per pass of w_from_gtg_kernel (at most)
constexpr int kWRows = 256;  // pattern rows per workgroup of w_band_kernel
constexpr int kWDeg = 16;    // most entries per pattern row that w_band_kernel holds
constexpr int kWPassBytes = 64 * 1024;  // LDS of one w_band_kernel pass (k x cb x band doubles)
// W_t = B_t Y as w_from_gtg_kernel, for patterns with at most kWDeg entries per row; KF >= the
// models' k.  Grid: x over tiles of kWRows pattern rows, y over slices of cs columns, z as in
// w_from_gtg_kernel; dynamic LDS k * cb * (widest band) doubles.
template <int KF>
__global__ void w_band_kernel(const Models Ms, int t, int zdiv, const int32_t* zn,
                              const double* Y, long long zY, double* W, long long zW,
                              const double* phi, int cb, int cs);
// zdiv > 0: grid.z runs over (chain, block) pairs, z = chain * zdiv + block (t is then the
// block, zY and zW block strides, and blocks at or past zn[chain] are skipped; zn may be null)
__global__ void w_from_gtg_kernel(const Models Ms, int t, int zdiv, const int32_t* zn,
                                  const double* Y, long long zY, double* W, long long zW,
                                  const double* phi, int cb);
__global__ void fd_hessian_kernel(const double* fv, int d, double h, double* f, double* H);
__global__ void grad_hessian_kernel(const double* fv, const double* gv, int d, double h,
                                    double* f, double* grad, double* H);

}  // namespace adelia
