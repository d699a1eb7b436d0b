// Uneven batch of independent BTA factorisations (Alg. 1 over many matrices at once).
//
// Matrices are grouped by block size b.  A group is packed into uniform-stride chains (the
// layout every sweep kernel takes): n_max block slots, arrows padded to the group's largest a
// with identity tip rows (they add log 1 = 0 to the log-determinant and leave the real rows'
// arithmetic unchanged), the right-hand side as the last arrow row.  One sweep then runs the
// whole group; at step i a chain with n_z <= i takes no part (the kernels read the per-chain
// block counts), and the B block after a chain's last block is zero, so its final TRMM and
// Schur update touch only its arrow and tip.  Groups run one after another on the stream and
// reuse the same workspace.
#include <adelia.h>

#include <algorithm>
#include <climits>
#include <map>
#include <vector>

#include "common.h"
#include "internal_api.h"
#include "launchers.h"

using namespace adelia;

namespace {

// Results back to the callers' order.  A failing column in the tip was numbered after the
// group's n_max blocks; it is renumbered after the matrix's own n blocks.
__global__ void scatter_results_kernel(const double* ld, const int32_t* info, const int32_t* idx,
                                       const int32_t* zn, int nz, int nmax, int b, double* ld_out,
                                       int32_t* info_out) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= nz) return;
  ld_out[idx[z]] = ld[z];
  int32_t v = info[z];
  if (v == INT32_MAX) v = 0;
  else if (v > nmax * b) v -= (nmax - zn[z]) * b;
  info_out[idx[z]] = v;
}

struct Group {
  int b = 0, nmax = 0, amax = 0;
  std::vector<int> members;
};

struct GroupWs {
  double *D, *B, *G, *C, *LC, *T, *LBC, *S, *ldpart, *zsq, *ld, *Vp;
  int32_t *info, *cnt, *zn, *idx;
  long long zD, zB, zG, zC, zT, zLd;
  int ap, slotsB, npanel;
  size_t bytes;
};

GroupWs group_layout(const Group& g, bool rhs, char* base) {
  GroupWs w{};
  const int nz = (int)g.members.size();
  const long long bb = (long long)g.b * g.b;
  w.ap = g.amax + (rhs ? 1 : 0);
  const int apa = std::max(w.ap, 1);
  w.slotsB = std::max(1, g.nmax - 1);
  w.npanel = (g.b + kPanel - 1) / kPanel;
  size_t off = 0;
  auto take = [&](long long per_chain, long long& stride) {
    stride = per_chain;
    double* p = base ? reinterpret_cast<double*>(base + off) : nullptr;
    off = align_up(off + (size_t)per_chain * nz * sizeof(double));
    return p;
  };
  long long dummy;
  w.D = take((long long)g.nmax * bb, w.zD);
  w.B = take((long long)w.slotsB * bb, w.zB);
  w.G = take((long long)g.nmax * bb, w.zG);
  w.C = take((long long)g.nmax * apa * g.b, w.zC);
  w.LC = take((long long)g.nmax * apa * g.b, dummy);
  w.T = take((long long)apa * apa, w.zT);
  w.LBC = take((long long)(g.b + w.ap) * g.b, dummy);
  w.S = take(bb, dummy);
  w.ldpart = take((long long)g.nmax * w.npanel + 1, w.zLd);
  w.zsq = take(1, dummy);
  w.ld = take(1, dummy);
  w.Vp = take((long long)kPanel * kPanel, dummy);
  int32_t* ints = base ? reinterpret_cast<int32_t*>(base + off) : nullptr;
  off = align_up(off + (size_t)4 * nz * sizeof(int32_t));
  w.info = ints;
  w.cnt = ints ? ints + nz : nullptr;
  w.zn = ints ? ints + 2 * nz : nullptr;
  w.idx = ints ? ints + 3 * nz : nullptr;
  w.bytes = off;
  return w;
}

bool shape_ok(const adelia_bta_shape& sh) {
  if (sh.n < 1 || sh.b < 1 || sh.a < 0 || sh.a > 63 || sh.b > kMaxBlock) return false;
  const long long N = (long long)sh.n * sh.b + sh.a;
  return N <= INT_MAX && (long long)sh.n * sh.b <= INT_MAX;
}

std::vector<Group> make_groups(int count, const adelia_bta_shape* shapes) {
  std::map<int, Group> by_b;
  for (int i = 0; i < count; ++i) {
    Group& g = by_b[shapes[i].b];
    g.b = shapes[i].b;
    g.nmax = std::max(g.nmax, shapes[i].n);
    g.amax = std::max(g.amax, shapes[i].a);
    g.members.push_back(i);
  }
  std::vector<Group> out;
  for (auto& kv : by_b) out.push_back(kv.second);
  return out;
}

bool aligned8(const void* p) { return ((uintptr_t)p & 7) == 0; }

}  // namespace

extern "C" {

size_t adelia_bta_batched_workspace_bytes(int count, const adelia_bta_shape* shapes, int with_rhs) {
  if (count < 1 || !shapes) return 0;
  for (int i = 0; i < count; ++i)
    if (!shape_ok(shapes[i])) return 0;
  size_t need = 0;
  for (const Group& g : make_groups(count, shapes))
    need = std::max(need, group_layout(g, with_rhs != 0, nullptr).bytes);
  return need + 256;
}

int bta_factor_batched(adelia_ctx ctx, int count, const adelia_bta_shape* shapes,
                       double* const* D, double* const* B, double* const* C, double* const* T,
                       double* const* Dinv, double* const* rhs, double* logdet, int32_t* info,
                       void* ws, size_t ws_bytes, void* stream) {
  if (!ctx) return -1;
  if (count < 1 || !shapes) return -2;
  if (!D || !Dinv) return -3;
  for (int i = 0; i < count; ++i) {
    const adelia_bta_shape& sh = shapes[i];
    if (!shape_ok(sh)) return ADELIA_E_SHAPE;
    if (!D[i] || !aligned8(D[i]) || !Dinv[i] || !aligned8(Dinv[i])) return -3;
    if (sh.n > 1 && (!B || !B[i] || !aligned8(B[i]))) return -4;
    if (sh.a > 0 && (!C || !T || !C[i] || !aligned8(C[i]) || !T[i] || !aligned8(T[i]))) return -5;
    if (rhs && (!rhs[i] || !aligned8(rhs[i]))) return -8;
  }
  if (!logdet || !aligned8(logdet)) return -9;
  if (!info || ((uintptr_t)info & 3)) return -10;
  if (!ws || ((uintptr_t)ws & 255)) return -11;
  if (ws_bytes < adelia_bta_batched_workspace_bytes(count, shapes, rhs != nullptr))
    return ADELIA_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  const bool with_rhs = rhs != nullptr;
  char* base = reinterpret_cast<char*>(ws);
  int e = 0;
  for (const Group& g : make_groups(count, shapes)) {
    GroupWs w = group_layout(g, with_rhs, base);
    const int nz = (int)g.members.size(), b = g.b, ap = w.ap, amax = g.amax;
    const long long bb = (long long)b * b;
    // ---- pack
    e |= launch_fill_i32(w.info, nz, INT32_MAX, s);
    e |= launch_fill_i32(w.cnt, nz, 0, s);
    e |= launch_fill(w.ldpart, (long long)nz * w.zLd, 0.0, s);
    if (ap > 0) {
      e |= launch_fill(w.C, (long long)nz * w.zC, 0.0, s);
      e |= launch_fill(w.T, (long long)nz * w.zT, 0.0, s);
    }
    for (int z = 0; z < nz; ++z) {
      const int q = g.members[z];
      const int n = shapes[q].n, a = shapes[q].a;
      const long long nb = (long long)n * b;
      e |= launch_fill_i32(w.zn + z, 1, n, s);
      e |= launch_fill_i32(w.idx + z, 1, q, s);
      e |= launch_copy2d(D[q], b, 0, w.D + z * w.zD, b, 0, b, (int)nb, 1, s);
      if (n > 1) e |= launch_copy2d(B[q], b, 0, w.B + z * w.zB, b, 0, b, (int)(nb - b), 1, s);
      if (n < g.nmax) e |= launch_fill(w.B + z * w.zB + (long long)(n - 1) * bb, bb, 0.0, s);
      double* Cz = w.C + z * w.zC;
      double* Tz = w.T + z * w.zT;
      if (a > 0) {
        e |= launch_copy2d(C[q], a, 0, Cz, ap, 0, a, (int)nb, 1, s);
        e |= launch_copy2d(T[q], a, 0, Tz, ap, 0, a, a, 1, s);
      }
      if (amax > a) e |= launch_fill_strided(Tz + (long long)a * (ap + 1), ap + 1, amax - a, 1.0, s);
      if (with_rhs) {
        e |= launch_copy2d(rhs[q], 1, 0, Cz + amax, ap, 0, 1, (int)nb, 1, s);
        if (a > 0) e |= launch_copy2d(rhs[q] + nb, 1, 0, Tz + amax, ap, 0, 1, a, 1, s);
      }
    }
    if (e) return ADELIA_E_HIP;
    // ---- sweep
    BtaChains c{};
    c.n = g.nmax; c.b = b; c.a = amax; c.ap = ap; c.nz = nz;
    c.D = w.D; c.zD = w.zD; c.slotsD = g.nmax;
    c.Bin = w.B; c.zB = w.zB; c.slotsB = w.slotsB;
    c.LBC = w.LBC; c.zLBC = (long long)(b + ap) * b; c.slotsLBC = 1;
    c.C = w.C; c.zC = w.zC;
    c.T = w.T; c.zT = w.zT;
    c.G = w.G; c.zG = w.zG; c.slotsG = g.nmax;
    c.ldpart = w.ldpart; c.zLd = w.zLd;
    c.info = w.info;
    c.cnt = w.cnt;
    c.zn = w.zn;
    c.scratch = w.S; c.zS = bb;
    c.zsq = w.zsq;
    c.Vp = w.Vp; c.zVp = (long long)kPanel * kPanel;
    // with the context's streams: look-ahead steps, and each block's inverse on the side stream
    // (every block keeps its L_D and G slot), joined before the results are unpacked
    const bool side = ctx->has_streams;
    c.invert = !side;
    c.inv_maxwg = side ? ctx->side_maxwg : 0;
    Lookahead la = ctx->la;
    for (int i = 0; i < g.nmax; ++i) {
      if (bta_forward_block(c, i, s, side ? &la : nullptr)) return ADELIA_E_HIP;
      if (side && (hipEventRecord(ctx->fork[i % 3], s) != hipSuccess ||
                   hipStreamWaitEvent(ctx->s2, ctx->fork[i % 3], 0) != hipSuccess ||
                   bta_invert_block(c, i, ctx->s2)))
        return ADELIA_E_HIP;
      // [L_Bi; L_Ci] leave the one-block scratch for block i's slots
      if (i < g.nmax - 1 &&
          launch_copy2d(w.LBC, b + ap, c.zLBC, w.B + (long long)i * bb, b, w.zB, b, b, nz, s))
        return ADELIA_E_HIP;
      if (ap > 0 && launch_copy2d(w.LBC + b, b + ap, c.zLBC, w.LC + (long long)i * ap * b, ap,
                                  w.zC, ap, b, nz, s))
        return ADELIA_E_HIP;
    }
    if (side && (hipEventRecord(ctx->join, ctx->s2) != hipSuccess ||
                 hipStreamWaitEvent(s, ctx->join, 0) != hipSuccess))
      return ADELIA_E_HIP;
    if (bta_tip(c, s)) return ADELIA_E_HIP;
    e |= bta_logdet_reduce(w.ldpart, w.zLd, g.nmax * w.npanel + 1, w.ld, 1, nz, s);
    // ---- unpack
    for (int z = 0; z < nz; ++z) {
      const int q = g.members[z];
      const int n = shapes[q].n, a = shapes[q].a;
      const long long nb = (long long)n * b;
      e |= launch_copy2d(w.D + z * w.zD, b, 0, D[q], b, 0, b, (int)nb, 1, s);
      e |= launch_copy2d(w.G + z * w.zG, b, 0, Dinv[q], b, 0, b, (int)nb, 1, s);
      if (n > 1) e |= launch_copy2d(w.B + z * w.zB, b, 0, B[q], b, 0, b, (int)(nb - b), 1, s);
      const double* LCz = w.LC + z * w.zC;
      const double* Tz = w.T + z * w.zT;
      if (a > 0) {
        e |= launch_copy2d(LCz, ap, 0, C[q], a, 0, a, (int)nb, 1, s);
        e |= launch_copy2d(Tz, ap, 0, T[q], a, 0, a, a, 1, s);
      }
      if (with_rhs) {
        e |= launch_copy2d(LCz + amax, ap, 0, rhs[q], 1, 0, 1, (int)nb, 1, s);
        if (a > 0) e |= launch_copy2d(Tz + amax, ap, 0, rhs[q] + nb, 1, 0, 1, a, 1, s);
      }
      e |= launch_zero_upper(D[q], b, b, bb, n, 0, 1, s);
      e |= launch_zero_upper(Dinv[q], b, b, bb, n, 0, 1, s);
    }
    hipLaunchKernelGGL(scatter_results_kernel, dim3((nz + 255) / 256), dim3(256), 0, s, w.ld,
                       w.info, w.idx, w.zn, nz, g.nmax, b, logdet, info);
    if (hipGetLastError() != hipSuccess) e = 1;
    if (e) return ADELIA_E_HIP;
  }
  return 0;
}

}  // extern "C"
